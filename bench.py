#!/usr/bin/env python3
"""Throughput of the parallel-rejection KMC step for the 2D lattice Coulomb glass on one MI355X.

Workload: a batch of B independent samples (default 256, one workgroup per sample) at
L=128 (N=16384), half filling, W=1, xi=1, rc=10, T=0.02, E=0.005, Philox seed 3, sample ids
0..B-1, from the random initial configuration.  A step is one pass of the whole hot path
for every sample: `hops_per_step` accepted hops (proposal draw, occupancy filter,
Metropolis, lowest-accepted-label selection, hop execution, local-energy update) and, in
the FP32 form, the FP64 refresh that ends each refresh interval (default: the interval is
the step).  The timed region starts with every input resident in HBM.

The headline value is accepted hops/s of the FP32-with-FP64-refresh form; the plain FP64
form is timed on the same samples and reported beside it.  The JSON line also carries the
LDS roofline of the hop kernel (algorithmic bytes per launch / mean launch time from HIP
events on the library's stream) and the CPU oracle timed on this host.

Beside the headline (skipped with --no-legs, each guarded so that it cannot cost the
headline line): one sample of side 256 ... 2048 on the whole GPU at T = 0.05 (the paper's
large-lattice setting), one L = 64 sample at T = 0.001 and one simple cubic L = 16 sample at
T = 0.003 each with the label-parallel kernel and with one workgroup, the uneven batch (96
samples of L = 32 ... 160 run to simulated time 10^3) and a batch of simple cubic samples
(L = 16).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# LDS bandwidth of the chip: 256 CUs x 224 B/clk x 2.4 GHz, the best rate the unit probe
# (paper_1407_5026_amd/csrc/lds_probe.hip) measures on MI355X, with 16-byte ds_read_b128; 4-byte
# reads reach 65 B/clk (each LDS read instruction occupies the CU's LDS pipe for ~4-5 cycles
# whatever its width), and writes at most ~72 B/clk at any width
LDS_PEAK_GBS = 256 * 224 * 2.4
# LDS writes: the probe measures at most ~72 B/clk per CU with 8- or 16-byte stores
LDS_WRITE_BPC = 72.0
LDS_READ_BPC = 224.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_hops_fx_l128_b256_traffic.json")
KERNEL_SRCS = [os.path.join(ROOT, "paper_1407_5026_amd", "csrc", f) for f in ("hop_fx.hpp", "kernels.hpp", "layout.hpp")]
# the FP64 form's hop kernel: its own record, over its own sources
TRAFFIC_FILE64 = os.path.join(ROOT, "profiles", "k_hops_fx64_l128_b256_traffic.json")
KERNEL_SRCS64 = [os.path.join(ROOT, "paper_1407_5026_amd", "csrc", f)
                 for f in ("hop_fx64.hpp", "hop_fx.hpp", "kernels.hpp", "layout.hpp")]


def kernel_hash(srcs=None) -> str:
    """Hash of the hop kernel's sources: a traffic record applies only to the code it measured."""
    import hashlib

    h = hashlib.sha256()
    for p in (KERNEL_SRCS if srcs is None else srcs):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_record(kernel: str):
    """The committed counter record of a hop kernel (HBM bytes per launch from FETCH_SIZE
    and WRITE_SIZE scaled by a copy kernel of known size; VALU, SALU and LDS instructions per
    hop), or None when it was taken on another kernel instance or the kernel source has changed
    since."""
    path, srcs = (TRAFFIC_FILE64, KERNEL_SRCS64) if kernel.startswith("k_hops_fx64") else (TRAFFIC_FILE, KERNEL_SRCS)
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash(srcs) or not t.get("kernel", "").endswith(kernel):
        return None
    return t


def measured_traffic(kernel: str):
    t = counter_record(kernel)
    return None if t is None else t.get("bytes_per_launch")


def _cpu_worker(args):
    import oracle
    from workloads import headline

    b, warm, hops, seed = args
    s = headline(b + 1, seed=seed)[b]
    o = oracle.Oracle(L=s.L, n_e=s.n_e, W=s.W, xi=s.xi, rc=s.rc, T=s.T, E=s.E, seed=s.seed,
                      sample_id=s.sample_id)
    if warm:
        o.run(warm, log_cap=0)
    t0 = time.perf_counter()
    o.run(hops, log_cap=0)
    return hops, time.perf_counter() - t0


def host_cores() -> tuple[int, int]:
    """(cores the CPU leg uses, cores this process may run on).  The leg uses every core the
    process may run on, capped at the host share of one GPU (OMP_NUM_THREADS, 16 by default)."""
    nproc = len(os.sched_getaffinity(0))
    share = int(os.environ.get("OMP_NUM_THREADS", "16") or 16)
    return max(1, min(nproc, share)), nproc


def cpu_baseline(warm: int, hops: int, seed: int, cores: int, nproc: int) -> dict:
    """The serial FP64 oracle on this host: one headline sample per process, `warm` untimed hops
    from the random start (the GPU's warmup window), then `hops` timed hops; all processes run
    concurrently and the aggregate is the sum of their rates.  Called before this process
    touches the GPU (the worker processes are forked from it), and the pool is closed and
    joined, not terminated."""
    import multiprocessing as mp

    pool = mp.get_context("fork").Pool(cores)
    try:
        res = pool.map(_cpu_worker, [(b, warm, hops, seed) for b in range(cores)])
    finally:
        pool.close()
        pool.join()
    rate = sum(h / t for h, t in res)
    cpu_s = sum(t for _, t in res)
    return {"value": rate, "unit": "accepted hops/s", "cores": cores, "kind": "oracle", "host_nproc": nproc,
            "sample": f"serial FP64 oracle, L=128 T=0.02 E=0.005 rc=10, samples 0..{cores - 1}: "
                      f"hops {warm}..{warm + hops} of each sample timed after {warm} untimed hops from "
                      f"the random start, {cores} processes on a host where this process may use "
                      f"{nproc} cores, rates summed ({cpu_s:.1f} s of CPU time)"}


def run_form(cg, torch, samples, precision, args, hops_per_step):
    opts = cg.make_opts(precision=precision, M=args.M, block=args.block, K_refresh=args.K, clock_mode=args.clock)
    b = cg.Batch(samples, opts)
    n = len(samples)
    for _ in range(args.warmup):
        b.run_hops(hops_per_step)
    torch.cuda.synchronize()
    before = [b.stats(k) for k in range(n)]
    b.kernel_time()  # reset the event accumulators
    # window boundaries: events on the library's stream, read after the timed region
    per_win = max(1, args.window_hops // hops_per_step)
    marks = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        if k % per_win == 0:
            e = torch.cuda.Event(enable_timing=True)
            e.record(b.stream)
            marks.append((k, e))
        b.run_hops(hops_per_step)
    e = torch.cuda.Event(enable_timing=True)
    e.record(b.stream)
    marks.append((args.steps, e))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    windows = []
    for (k0, e0), (k1, e1) in zip(marks, marks[1:]):
        ms = e0.elapsed_time(e1)
        windows.append(n * hops_per_step * (k1 - k0) / (ms * 1e-3))
    hop_ms, hop_n, ref_ms, ref_n = b.kernel_time()
    after = [b.stats(k) for k in range(n)]
    hops = sum(a["hops"] - c["hops"] for a, c in zip(after, before))
    props = sum(a["s_last"] - c["s_last"] for a, c in zip(after, before))
    evald = sum(a["evaluated"] - c["evaluated"] for a, c in zip(after, before))
    theta = sum(a["theta_pass"] - c["theta_pass"] for a, c in zip(after, before))
    drift = max(a["max_drift"] for a in after)
    b.close()
    return dict(seconds=dt, hops=hops, proposals=props, evaluated=evald, theta=theta, hop_ms=hop_ms,
                hop_launches=hop_n, refresh_ms=ref_ms, refresh_launches=ref_n, max_drift=drift,
                windows=windows, window_hops=per_win * hops_per_step)


def lds_roofline(r: dict, N: int, s_eps: int, kernel: str) -> dict:
    """LDS roofline of a hop kernel from a timed run.  Algorithmic bytes per accepted hop: the
    update reads and writes the N energies (N s_eps each way); the proposals read 2 occupancy
    bytes per serial proposal plus two energies per evaluation that passes the occupancy
    filter (m_bar and theta_bar are the run's own).  `achieved` = bytes per hop x hops per
    launch / mean launch time (HIP events on the library's stream); `peak` = the best LDS read
    rate.  The same bytes against a read/write-split peak: reads at 224 B/clk, the N s_eps
    written bytes at 72 B/clk, so the split peak is (R + W) / (R / 224 + W / 72) B/clk per CU."""
    m_bar = r["proposals"] / max(r["hops"], 1)
    th_bar = r["theta"] / max(r["evaluated"], 1)
    write_b = N * s_eps
    read_b = N * s_eps + m_bar * (2 + th_bar * 2 * s_eps)
    bytes_per_hop = read_b + write_b
    per_launch_hops = r["hops"] / max(r["hop_launches"], 1)
    mean_launch_s = r["hop_ms"] / max(r["hop_launches"], 1) * 1e-3
    achieved = bytes_per_hop * per_launch_hops / mean_launch_s / 1e9
    split_bpc = bytes_per_hop / (read_b / LDS_READ_BPC + write_b / LDS_WRITE_BPC)
    split_peak = 256 * split_bpc * 2.4
    return {"bound": "lds", "achieved": achieved, "peak": LDS_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / LDS_PEAK_GBS, "traffic": measured_traffic(kernel), "kernel": kernel,
            "bytes_per_hop": bytes_per_hop, "read_bytes_per_hop": read_b, "write_bytes_per_hop": write_b,
            "hops_per_launch": per_launch_hops, "mean_launch_ms": mean_launch_s * 1e3,
            "peak_rw_split": split_peak, "frac_rw_split": achieved / split_peak}


def phase_split(cg, torch, samples, args) -> dict:
    """The paper's split of the time per executed hop into the rejection part W_R (drawing,
    evaluating and selecting labels) and the update part W_U (step 3b): the headline batch in
    the FP32 form with the phase-timer instance of the hop kernel (wave 0's shader cycles per
    phase), one untimed step from the random start, then `args.phase_steps` steps."""
    opts = cg.make_opts(precision=cg.CG_FP32_REFRESH, M=args.M, block=args.block, K_refresh=args.K,
                        clock_mode=args.clock, phase_timers=1)
    b = cg.Batch(samples, opts)
    n = len(samples)
    b.run_hops(args.hops_per_step)
    torch.cuda.synchronize()
    before = [b.stats(k) for k in range(n)]
    b.kernel_time()
    for _ in range(args.phase_steps):
        b.run_hops(args.hops_per_step)
    torch.cuda.synchronize()
    hop_ms, hop_n, _, _ = b.kernel_time()
    after = [b.stats(k) for k in range(n)]
    b.close()
    hops = sum(a["hops"] - c["hops"] for a, c in zip(after, before))
    cyc = [sum(a["phase_cycles"][i] - c["phase_cycles"][i] for a, c in zip(after, before)) / hops for i in range(4)]
    total = sum(cyc)
    # per-sample time per hop: every sample runs on its own CU for the whole launch
    us_hop = hop_ms * 1e3 / (hops / n)
    wr = (cyc[0] + cyc[1] + cyc[2]) / total
    return {"kernel_instance": "phase timers", "hops_per_sample": hops // n,
            "cycles_per_hop": {"draw": cyc[0], "evaluate": cyc[1], "select_and_execute": cyc[2],
                               "update": cyc[3]},
            "us_per_hop_per_sample": us_hop, "W_R_us": wr * us_hop, "W_U_us": (1 - wr) * us_hop,
            "W_R_frac": wr}


def batched_l64(cg, torch, hops: int, step: int) -> dict:
    """256 samples at L = 64, rc = 8, E = 0.01, T round-robin over {0.02, 0.03, 0.05, 0.08, 0.12},
    FP32 form, M = 2048, refresh every 2048 hops: `hops` accepted hops per sample from the
    random start in steps of `step`."""
    from workloads import batched_l64 as recipe

    samples = recipe(256)
    b = cg.Batch(samples, cg.make_opts(precision=cg.CG_FP32_REFRESH, M=2048, K_refresh=2048))
    torch.cuda.synchronize()
    b.kernel_time()
    t0 = time.perf_counter()
    done = 0
    while done < hops:
        n = min(step, hops - done)
        b.run_hops(n)
        done += n
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    hop_ms, hop_n, ref_ms, ref_n = b.kernel_time()
    st = [b.stats(k) for k in range(len(samples))]
    b.close()
    by_T = {}
    for smp, x in zip(samples, st):
        by_T.setdefault(smp.T, []).append(x["s_last"] / max(x["hops"], 1))
    return {"samples": len(samples), "L": 64, "hops_per_sample": hops, "M": 2048, "K_refresh": 2048,
            "seconds": dt, "hops_per_s": sum(x["hops"] for x in st) / dt, "hop_kernel_ms": hop_ms,
            "refresh_ms": ref_ms, "max_drift": max(x["max_drift"] for x in st),
            "m_bar_by_T": {str(T): sum(v) / len(v) for T, v in sorted(by_T.items())}}


def large_lattice(cg, torch, L: int, hops: int, warm: int, T: float, variant: int = 0, spread: int = 0,
                  M: int = 0, dim: int = 2) -> dict:
    """One sample of side L on the whole GPU (FP64 form): the paper's large-lattice setting
    (nu = 1/2, xi = 1, W = 1, E = T/10; hop cutoff rc = 10, 6 at L = 16), warm untimed hops from the random
    start, then `hops` timed hops.  Per hop the update writes the N FP64 energies of the
    proposals' mirror (8 N bytes) and reads two FP64 inverse distances per site from the
    (|dy|, |dx|) table (16 N bytes, cache-resident for L <= 2048).  variant 6: the
    label-parallel kernel (a replica of the sample on each of `spread` workgroups, 0 = every CU;
    rounds of spread x M labels, M = 1024 or 2048 per workgroup)."""
    from workloads import Sample

    N = L ** 3 if dim == 3 else L * L
    rc = 4.0 if dim == 3 else (10.0 if L >= 32 else 6.0)  # the hop cutoff stays below L/2
    s = Sample(L, N // 2, 1.0, 1.0, rc, T, T / 10, 7, 0, dim=dim)
    t0 = time.perf_counter()
    b = cg.Batch([s], cg.make_opts(precision=cg.CG_FP64, variant=variant, spread=spread, M=M,
                                   max_labels_per_call=1 << 40))
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t0
    if warm:
        b.run_hops(warm)
    torch.cuda.synchronize()
    st0 = b.stats(0)
    b.kernel_time()
    t0 = time.perf_counter()
    b.run_hops(hops)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    hop_ms, hop_n, _, _ = b.kernel_time()
    st1 = b.stats(0)
    done = max(st1["hops"] - st0["hops"], 1)
    m_bar = (st1["s_last"] - st0["s_last"]) / done
    rounds = (st1["rounds"] - st0["rounds"]) / done
    b.close()
    paper = None if dim == 3 else {0.05: {"64": 0.10, "2048": 1.04}, 0.001: {"64": 0.27, "2048": 1.23}}.get(T, {}).get(str(L))
    us = hop_ms * 1e3 / done
    if dim == 3:
        kernel = "k_hops_wide3" if variant == 6 else "k_hops3 (one workgroup)"
    elif variant == 6:
        kernel = "k_hops_wide"
    elif L > 192:
        kernel = "k_hops_big"
    else:
        kernel = "k_hops_fx64 (one workgroup)" if L in (64, 128) else "k_hops (one workgroup)"
    return {"L": L, "dim": dim, "N": N, "rc": rc, "T": T, "E": T / 10, "kernel": kernel, "spread": spread, "M": M or 1024, "hops": hops, "warmup_hops": warm,
            "hops_per_s": hops / dt, "us_per_hop": dt / hops * 1e6, "kernel_us_per_hop": us,
            "kernel_launches": hop_n, "m_bar": m_bar, "rounds_per_hop": rounds,
            "update_bytes_per_hop": 24 * N, "update_GBps": 24 * N / (us * 1e-6) / 1e9,
            "init_s": init_s, "paper_gpu_ms_per_hop": paper}


def uneven(cg, torch, n: int, t_end: float) -> dict:
    """The uneven batch: n samples with L drawn from {32, 48, 64, 96, 128, 160} and per-sample
    T, E and W (rc = 10), FP32 form with the kernel's chunk, the refresh period and each
    sample's PR width M* = min(1/A, 16384) autotuned, every sample run from the random start to
    simulated time t_end.  Every lattice's FP32 values fit LDS (L <= 160); the samples finish at
    different hop counts."""
    import dataclasses

    from workloads import uneven_batch

    samples = uneven_batch(n)
    t0 = time.perf_counter()
    opts, widths = cg.autotune(samples, cg.make_opts(precision=cg.CG_FP32_REFRESH), widths=True)
    tune_s = time.perf_counter() - t0
    samples = [dataclasses.replace(s, M=w) for s, w in zip(samples, widths)]
    b = cg.Batch(samples, opts)
    torch.cuda.synchronize()
    b.kernel_time()
    t0 = time.perf_counter()
    b.run_time(t_end)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    hop_ms, hop_n, ref_ms, ref_n = b.kernel_time()
    st = [b.stats(k) for k in range(n)]
    b.close()
    hops = sum(x["hops"] for x in st)
    by_L, M_by_L = {}, {}
    for s, x in zip(samples, st):
        by_L.setdefault(s.L, []).append(x["hops"])
        M_by_L.setdefault(s.L, []).append(s.M)
    return {"samples": n, "t_end": t_end, "chunk": opts.M, "K_refresh": opts.K_refresh, "hops": hops,
            "seconds": dt, "hops_per_s": hops / dt, "hop_kernel_ms": hop_ms, "hop_launches": hop_n,
            "refresh_ms": ref_ms, "max_drift": max(x["max_drift"] for x in st), "autotune_s": tune_s,
            "mean_hops_by_L": {str(L): round(sum(v) / len(v)) for L, v in sorted(by_L.items())},
            "M_by_L": {str(L): sorted(set(v)) for L, v in sorted(M_by_L.items())},
            "mean_p_per_hop": sum(x["sum_p"] for x in st) / max(hops, 1)}


def cubic(cg, torch, L: int, batch: int, hops: int, steps: int) -> dict:
    """Batch of simple cubic samples (FP64 form; nu = 1/2, W = 1, xi = 1, rc = 4, T = 0.05,
    E = 0.005) from the random start: one untimed step of `hops` hops per sample, then `steps`
    timed steps; beside it the 3D oracle on one sample of the batch, single core."""
    import oracle
    from workloads import Sample

    samples = [Sample(L, L ** 3 // 2, 1.0, 1.0, 4.0, 0.05, 0.005, 13, b, dim=3) for b in range(batch)]
    b = cg.Batch(samples, cg.make_opts(precision=cg.CG_FP64))
    b.run_hops(hops)
    torch.cuda.synchronize()
    b.kernel_time()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.run_hops(hops)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    hop_ms, hop_n, _, _ = b.kernel_time()
    st = [b.stats(k) for k in range(batch)]
    b.close()
    s = samples[0]
    o = oracle.Oracle3D(L=L, n_e=s.n_e, W=s.W, xi=s.xi, rc=s.rc, T=s.T, E=s.E, seed=s.seed, sample_id=0)
    o.run(hops)
    n_cpu = max(64, hops // 8)
    c0 = time.perf_counter()
    o.run(n_cpu)
    cpu = n_cpu / (time.perf_counter() - c0)
    m_bar = sum(x["s_last"] for x in st) / sum(x["hops"] for x in st)
    return {"L": L, "N": L ** 3, "batch": batch, "rc": 4.0, "T": 0.05, "E": 0.005, "hops_per_step": hops,
            "steps": steps, "hops_per_s": batch * hops * steps / dt, "mean_launch_ms": hop_ms / max(hop_n, 1),
            "m_bar": m_bar, "cpu_oracle_one_core_hops_per_s": cpu,
            "cpu_sample": f"3D oracle, sample 0, hops {hops}..{hops + n_cpu} after {hops} untimed"}


def pair_hops(cg, torch, batch: int, pair: float, hops: int, steps: int) -> dict:
    """Pair hops (a label proposes two electrons moving at once with probability `pair`: the
    multi-electron extension of sections "Code performance" and "Conclusions"): the headline
    parameters in the FP64 form from the random start, one untimed step of `hops` hops per
    sample, then `steps` timed steps, on the pair-hop kernel; beside it the same batch with
    single hops only on the generic FP64 kernel it derives from (variant 1)."""
    import dataclasses

    from workloads import headline

    out = {"batch": batch, "L": 128, "T": 0.02, "pair_probability": pair, "hops_per_step": hops, "steps": steps}
    for key, p, variant in (("pair", pair, 0), ("single", 0.0, 1)):
        samples = [dataclasses.replace(s, pair=p) for s in headline(batch)]
        b = cg.Batch(samples, cg.make_opts(precision=cg.CG_FP64, variant=variant))
        b.run_hops(hops)
        torch.cuda.synchronize()
        s0 = [b.stats(k) for k in range(batch)]
        b.kernel_time()
        t0 = time.perf_counter()
        for _ in range(steps):
            b.run_hops(hops)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        hop_ms, hop_n, _, _ = b.kernel_time()
        s1 = [b.stats(k) for k in range(batch)]
        b.close()
        n_h = sum(x["hops"] - y["hops"] for x, y in zip(s1, s0))
        out[key] = {"hops_per_s": n_h / dt, "mean_launch_ms": hop_ms / max(hop_n, 1),
                    "m_bar": sum(x["s_last"] - y["s_last"] for x, y in zip(s1, s0)) / max(n_h, 1),
                    "rounds_per_hop": sum(x["rounds"] - y["rounds"] for x, y in zip(s1, s0)) / max(n_h, 1)}
    out["pair"]["kernel"] = "k_hops_pair<true, 2, 8, true>"
    out["single"]["kernel"] = "k_hops<double, 1, true, 2, 8, true, kModeLds>"
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    # default: 10^6 accepted hops per sample from the random start (one untimed step of 4096
    # hops, then 244 timed steps), reported whole-run and per window of ~10^5 hops
    ap.add_argument("--steps", type=int, default=244)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--window-hops", type=int, default=98304)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--hops-per-step", type=int, default=4096)
    ap.add_argument("--M", type=int, default=8192)
    ap.add_argument("--block", type=int, default=1024)
    ap.add_argument("--K", type=int, default=4096)
    ap.add_argument("--clock", type=int, default=0,
                    help="clock mode: 0 deterministic m/Gamma (default), 1 Gaussian, 2 exact Gamma(m)")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--cpu-hops", type=int, default=8192)
    ap.add_argument("--cpu-cores", type=int, default=0)
    ap.add_argument("--skip-cpu", action="store_true")
    # legs beside the headline (single samples on the whole GPU, the cubic lattice); each is
    # guarded so that it can never cost the headline line
    ap.add_argument("--no-legs", action="store_true", help="time the headline workload only")
    ap.add_argument("--large-L", type=int, nargs="*", default=[256, 512, 1024, 2048],
                    help="time one sample of each of these sides (powers of two, 256..2048) on the "
                         "whole GPU, FP64, at --large-T")
    ap.add_argument("--large-hops", type=int, default=8000)
    ap.add_argument("--large-T", type=float, default=0.05)
    ap.add_argument("--wide-L", type=int, nargs="*", default=[64],
                    help="time one sample of each of these sides (powers of two, 16..128) with the "
                         "label-parallel kernel (variant 6) and with one workgroup, at --wide-T, FP64")
    ap.add_argument("--wide-T", type=float, default=0.001)
    ap.add_argument("--wide-spread", type=int, default=128, help="workgroups per sample of the label-parallel "
                                                                   "kernel (0 = every CU)")
    ap.add_argument("--wide-M", type=int, default=2048, help="labels per workgroup and round (1024 or 2048)")
    ap.add_argument("--wide3-L", type=int, nargs="*", default=[16],
                    help="time one simple cubic sample of each of these sides (<= 24) with the label-parallel "
                         "kernel and with one workgroup, at --wide3-T, FP64")
    ap.add_argument("--wide3-T", type=float, default=0.003)
    ap.add_argument("--uneven", type=int, default=96,
                    help="time the uneven batch of this many samples to --uneven-t (0 = none)")
    ap.add_argument("--uneven-t", type=float, default=1000.0)
    ap.add_argument("--cubic-L", type=int, default=16,
                    help="time a batch of simple cubic samples of this side (FP64 form; 0 = none)")
    ap.add_argument("--cubic-hops", type=int, default=2048)
    ap.add_argument("--cubic-steps", type=int, default=20)
    ap.add_argument("--l64-hops", type=int, default=200_000,
                    help="hops per sample of the 256-sample L = 64 temperature-grid batch (0 = none)")
    ap.add_argument("--pair", type=float, default=0.1,
                    help="pair-hop probability of the pair-hop leg (FP64, headline parameters; 0 = none)")
    ap.add_argument("--pair-steps", type=int, default=5)
    ap.add_argument("--legs", nargs="*", default=None,
                    help="run only these legs: l64 large wide wide3 uneven cubic pair (default: all)")
    ap.add_argument("--phase-steps", type=int, default=4,
                    help="steps of the phase-timer run that splits a hop into W_R and W_U (0 = none)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before timing, copy this many MiB with a plain device copy (a counter "
                         "calibration point for FETCH_SIZE / WRITE_SIZE runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (samples are independent; a batch would split across "
              f"GPUs without communication); --gpus {args.gpus} is not supported", file=sys.stderr)
        return 2

    from workloads import headline

    cpu = None
    if not args.skip_cpu:
        # before this process touches the GPU: the oracle's worker processes are forked from it
        cores, nproc = host_cores()
        if args.cpu_cores:
            cores = args.cpu_cores
        print(f"[bench] CPU oracle on {cores} cores ({nproc} available)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.warmup * args.hops_per_step, args.cpu_hops, headline(1)[0].seed, cores, nproc)
        print(f"[bench] CPU oracle done: {cpu['value']:.4g} hops/s", file=sys.stderr, flush=True)

    import torch

    import paper_1407_5026_amd as cg

    cg.load()
    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", "0")))
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {n} bytes done", file=sys.stderr, flush=True)
        del src, dst
    samples = headline(args.batch)
    N = samples[0].L ** 2
    print(f"[bench] FP32+refresh: B={args.batch} L=128 hops/step={args.hops_per_step} "
          f"steps={args.steps} warmup={args.warmup} M={args.M} block={args.block} K={args.K}",
          file=sys.stderr, flush=True)
    r32 = run_form(cg, torch, samples, cg.CG_FP32_REFRESH, args, args.hops_per_step)
    print(f"[bench] FP32 done: {r32['hops'] / r32['seconds']:.4g} hops/s", file=sys.stderr, flush=True)
    r64 = None
    if not args.skip_fp64:
        r64 = run_form(cg, torch, samples, cg.CG_FP64, args, args.hops_per_step)
        print(f"[bench] FP64 done: {r64['hops'] / r64['seconds']:.4g} hops/s", file=sys.stderr, flush=True)

    value = r32["hops"] / r32["seconds"]
    kernel = f"k_hops_fx<128, {1 if args.M <= 1024 else 2}, {0 if args.clock == 0 else 1}, 16, false>"
    out = {
        "metric": "accepted hops/s per GPU (L=128, T=0.02, batched) FP32+refresh vs FP64 PR",
        "value": value,
        "unit": "accepted hops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["seconds"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.batch} samples L=128 N=16384 half filling W=1 xi=1 rc=10 "
                               f"T=0.02 E=0.005 from the random start: {args.warmup * args.hops_per_step} "
                               f"untimed then {args.steps * args.hops_per_step} timed accepted hops per "
                               f"sample in steps of {args.hops_per_step}, FP32 with FP64 refresh every "
                               f"{args.K} hops",
                   "batch": args.batch, "L": 128, "M": args.M, "block": args.block,
                   "K_refresh": args.K, "hops_per_step": args.hops_per_step, "clock_mode": args.clock},
        "proposals_per_s": r32["proposals"] / r32["seconds"],
        "evaluated_labels_per_s": r32["evaluated"] / r32["seconds"],
        "fp32_max_drift": r32["max_drift"],
        "refresh_ms_per_step": r32["refresh_ms"] / args.steps,
        "window_hops_per_sample": r32["window_hops"],
        "fp32_window_hops_per_s": [round(v) for v in r32["windows"]],
        "roofline": lds_roofline(r32, N, 4, kernel),
    }
    rec = counter_record(kernel)
    if rec is not None and "valu_insts_per_hop" in rec:
        # VALU issue fraction: wave instructions per hop (counter run, the 41st launch: hops
        # 163840..167936 of each sample) x this run's hops/s, against 256 CUs x 1.7 wave
        # instructions per clock (the probe's FP32 rate) x 2.4 GHz
        out["valu_frac"] = rec["valu_insts_per_hop"] * value / (256 * 1.7 * 2.4e9)
        out["lds_insts_per_hop"] = rec["lds_insts_per_hop"]
    if r64 is not None:
        out["fp64_value"] = r64["hops"] / r64["seconds"]
        out["fp64_window_hops_per_s"] = [round(v) for v in r64["windows"]]
        out["fp64_ms_per_step"] = r64["seconds"] / args.steps * 1e3
        out["roofline_fp64"] = lds_roofline(r64, N, 8, "k_hops_fx64<128, 1, 0>")
    def leg(name, fn):
        print(f"[bench] {name}", file=sys.stderr, flush=True)
        try:
            return fn()
        except Exception as e:  # reported in the line; the headline stands
            print(f"[bench] {name} failed: {e!r}", file=sys.stderr, flush=True)
            return {"error": repr(e)}

    if args.phase_steps:
        out["phase_split_fp32"] = leg("phase timers (W_R / W_U per hop)",
                                      lambda: phase_split(cg, torch, samples, args))
    if not args.no_legs:
        want = (lambda name: True) if args.legs is None else (lambda name: name in args.legs)
        if not want("l64"):
            args.l64_hops = 0
        if not want("large"):
            args.large_L = []
        if not want("wide"):
            args.wide_L = []
        if not want("wide3"):
            args.wide3_L = []
        if not want("uneven"):
            args.uneven = 0
        if not want("cubic"):
            args.cubic_L = 0
        if not want("pair"):
            args.pair = 0.0
        if args.l64_hops:
            out["batched_l64_fp32"] = leg(f"256 samples L=64 over the T grid, {args.l64_hops} hops each",
                                          lambda: batched_l64(cg, torch, args.l64_hops, 8192))
        if args.large_L:
            out["large_lattice_fp64"] = [
                leg(f"whole-GPU sample L={L} T={args.large_T}",
                    lambda L=L: large_lattice(cg, torch, L, args.large_hops, args.large_hops // 4, args.large_T))
                for L in args.large_L]
        if args.wide_L:
            out["label_parallel_fp64"] = []
            for L in args.wide_L:
                for variant in (6, 0):
                    out["label_parallel_fp64"].append(
                        leg(f"single sample L={L} T={args.wide_T} variant {variant}",
                            lambda L=L, v=variant: large_lattice(cg, torch, L, args.large_hops, args.large_hops // 4,
                                                                 args.wide_T, variant=v, spread=args.wide_spread if v else 0,
                                                                 M=args.wide_M if v else 0)))
        if args.wide3_L:
            out["label_parallel_cubic_fp64"] = []
            for L in args.wide3_L:
                for variant in (6, 0):
                    out["label_parallel_cubic_fp64"].append(
                        leg(f"single cubic sample L={L} T={args.wide3_T} variant {variant}",
                            lambda L=L, v=variant: large_lattice(cg, torch, L, args.large_hops, args.large_hops // 4,
                                                                 args.wide3_T, variant=v,
                                                                 spread=args.wide_spread if v else 0, dim=3)))
        if args.uneven:
            out["uneven_batch_fp32"] = leg(f"uneven batch of {args.uneven} samples to t={args.uneven_t}",
                                           lambda: uneven(cg, torch, args.uneven, args.uneven_t))
        if args.cubic_L:
            out["cubic_fp64"] = leg(f"cubic batch L={args.cubic_L}",
                                    lambda: cubic(cg, torch, args.cubic_L, args.batch, args.cubic_hops, args.cubic_steps))
        if args.pair > 0:
            out["pair_hops_fp64"] = leg(f"pair hops p={args.pair} L=128",
                                        lambda: pair_hops(cg, torch, args.batch, args.pair, args.hops_per_step,
                                                          args.pair_steps))
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
