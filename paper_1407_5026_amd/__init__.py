"""Python binding of libcgkmc: parallel-rejection kinetic Monte Carlo of the 2D lattice
Coulomb glass on MI355X (gfx950).

Argument marshalling only.  Every step of the simulation runs in the library's HIP
kernels (see ``include/cgkmc.h`` for the C ABI this module mirrors function by
function).  PyTorch supplies device memory (the arena) and the HIP stream.  If the
built library is missing this module raises at import of the library, it has no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcgkmc.so")

CG_OK = 0
CG_EINVAL = -1
CG_ENOSPC = -2
CG_EHIP = -3
CG_ESTALL = -4

CG_FP64 = 0
CG_FP32_REFRESH = 1
CG_CLOCK_DET = 0
CG_CLOCK_GAUSS = 1
CG_CLOCK_GAMMA = 2

EXPORTS = (
    "cg_arena_bytes", "cg_create", "cg_destroy", "cg_run_hops", "cg_run_time", "cg_refresh",
    "cg_set_TE", "cg_get_occupation", "cg_get_local_energies", "cg_get_phi", "cg_get_stats",
    "cg_get_clock", "cg_get_current", "cg_get_hop_log", "cg_take_kernel_time", "cg_autotune", "cg_last_error",
    "cg_save", "cg_load", "cg_dos", "cg_dos_noalloc",
)


class cg_sample_desc(C.Structure):
    _fields_ = [("L", C.c_int32), ("n_electrons", C.c_int32), ("W", C.c_double), ("xi", C.c_double),
                ("rc", C.c_double), ("T", C.c_double), ("E", C.c_double), ("seed", C.c_uint64),
                ("sample_id", C.c_uint32), ("dim", C.c_int32), ("pair", C.c_double), ("M", C.c_int32)]


class cg_run_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("M", C.c_int32), ("block", C.c_int32),
                ("K_refresh", C.c_int32), ("clock_mode", C.c_int32), ("log_hops", C.c_int32),
                ("phase_timers", C.c_int32), ("use_graph", C.c_int32), ("variant", C.c_int32),
                ("spread", C.c_int32), ("max_labels_per_call", C.c_uint64)]


class cg_stats(C.Structure):
    _fields_ = [("hops", C.c_uint64), ("s_last", C.c_uint64), ("s_scan", C.c_uint64), ("P", C.c_int64),
                ("t", C.c_double), ("H0", C.c_double), ("sum_p", C.c_uint64), ("rounds", C.c_uint64),
                ("evaluated", C.c_uint64), ("theta_pass", C.c_uint64), ("refreshes", C.c_uint64),
                ("max_drift", C.c_double), ("last_drift", C.c_double), ("status", C.c_int32),
                ("since_refresh", C.c_int32), ("logged", C.c_int64),
                ("phase_cycles", C.c_uint64 * 4)]


class CgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libcgkmc error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libcgkmc.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() or "
                          f"python paper_1407_5026_amd/build.py")
    try:  # bind to the HIP runtime torch already loaded (same soname) when torch is present
        import torch  # noqa: F401
    except Exception:
        pass
    L = C.CDLL(path, mode=C.RTLD_GLOBAL)
    P = C.POINTER
    vp = C.c_void_p
    L.cg_arena_bytes.argtypes = [P(cg_sample_desc), C.c_int32, P(cg_run_opts), P(C.c_size_t)]
    L.cg_create.argtypes = [P(vp), P(cg_sample_desc), C.c_int32, P(cg_run_opts), vp, C.c_size_t, vp]
    L.cg_destroy.argtypes = [vp]
    L.cg_run_hops.argtypes = [vp, C.c_int64]
    L.cg_run_time.argtypes = [vp, C.c_double]
    L.cg_refresh.argtypes = [vp]
    L.cg_set_TE.argtypes = [vp, C.c_int32, C.c_double, C.c_double]
    L.cg_get_occupation.argtypes = [vp, C.c_int32, P(C.c_uint8)]
    L.cg_get_local_energies.argtypes = [vp, C.c_int32, P(C.c_double)]
    L.cg_get_phi.argtypes = [vp, C.c_int32, P(C.c_double)]
    L.cg_get_stats.argtypes = [vp, C.c_int32, P(cg_stats)]
    L.cg_get_clock.argtypes = [vp, C.c_int32, P(C.c_double)]
    L.cg_get_current.argtypes = [vp, C.c_int32, P(C.c_double), P(C.c_int64), P(C.c_double)]
    L.cg_get_hop_log.argtypes = [vp, C.c_int32, P(C.c_uint64), P(C.c_int32), P(C.c_int32), C.c_int64,
                                 P(C.c_int64)]
    L.cg_dos.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32, P(C.c_uint64),
                         P(C.c_uint64), P(C.c_uint64)]
    L.cg_dos_noalloc.argtypes = L.cg_dos.argtypes
    L.cg_save.argtypes = [vp, C.c_int32, vp, P(C.c_size_t)]
    L.cg_load.argtypes = [vp, C.c_int32, vp, C.c_size_t]
    L.cg_take_kernel_time.argtypes = [vp, P(C.c_double), P(C.c_int64), P(C.c_double), P(C.c_int64)]
    L.cg_autotune.argtypes = [P(cg_sample_desc), C.c_int32, P(cg_run_opts), vp, C.c_size_t, vp, C.c_int64,
                              C.c_double, P(C.c_int32)]
    L.cg_last_error.restype = C.c_char_p
    for f in EXPORTS:
        if f != "cg_last_error":
            getattr(L, f).restype = C.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != CG_OK:
        raise CgError(rc, load().cg_last_error().decode())


def _descs(samples):
    arr = (cg_sample_desc * len(samples))()
    for k, s in enumerate(samples):
        d = s if isinstance(s, dict) else s.as_dict()
        arr[k] = cg_sample_desc(int(d["L"]), int(d.get("n_e", d.get("n_electrons"))), float(d["W"]),
                                float(d["xi"]), float(d["rc"]), float(d["T"]), float(d["E"]),
                                int(d["seed"]), int(d["sample_id"]), int(d.get("dim", 2)),
                                float(d.get("pair", 0.0)), int(d.get("M", 0)))
    return arr


def make_opts(precision=CG_FP64, M=0, block=0, K_refresh=0, clock_mode=CG_CLOCK_DET, log_hops=0,
              max_labels_per_call=0, phase_timers=0, use_graph=0, variant=0, spread=0) -> cg_run_opts:
    return cg_run_opts(precision, M, block, K_refresh, clock_mode, log_hops, phase_timers, use_graph,
                       variant, spread, max_labels_per_call)


def arena_bytes(samples, opts: cg_run_opts) -> int:
    d = _descs(samples)
    n = C.c_size_t()
    _check(load().cg_arena_bytes(d, len(samples), C.byref(opts), C.byref(n)))
    return n.value


def autotune(samples, opts: cg_run_opts, trial_hops: int = 2048, drift_target: float = 1e-5,
             device="cuda", widths: bool = False):
    """Tuned copy of `opts` (chunk width M and, in the FP32 form, refresh period K) from short
    trial runs of these samples in a scratch arena; with widths=True also each sample's PR
    width min(1/A, 16384) as a power of two >= 512: returns (opts, [M per sample])."""
    import torch

    lib = load()
    d = _descs(samples)
    nbytes = arena_bytes(samples, opts)
    arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    ptr = (arena.data_ptr() + 255) & ~255
    out = cg_run_opts.from_buffer_copy(opts)
    stream = torch.cuda.current_stream(arena.device)
    w = (C.c_int32 * len(samples))() if widths else None
    _check(lib.cg_autotune(d, len(samples), C.byref(out), C.c_void_p(ptr), nbytes,
                           C.c_void_p(stream.cuda_stream), int(trial_hops), float(drift_target), w))
    del arena
    return (out, list(w)) if widths else out


class Batch:
    """A batch of samples living in one device arena (a torch uint8 tensor)."""

    def __init__(self, samples, opts: cg_run_opts | None = None, device="cuda", stream=None):
        import torch

        lib = load()
        self.samples = list(samples)
        self.opts = opts if opts is not None else make_opts()
        self.n = len(self.samples)
        self._descs = _descs(self.samples)
        nbytes = arena_bytes(self.samples, self.opts)
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        ptr = self.arena.data_ptr()
        self._arena_ptr = (ptr + 255) & ~255
        if stream is None:
            # graph replay cannot capture the legacy default stream: give the batch its own
            stream = (torch.cuda.Stream(self.arena.device) if self.opts.use_graph
                      else torch.cuda.current_stream(self.arena.device))
        self.stream = stream
        self.N = [int(d.L) ** (3 if d.dim == 3 else 2) for d in self._descs]
        h = C.c_void_p()
        _check(lib.cg_create(C.byref(h), self._descs, self.n, C.byref(self.opts),
                             C.c_void_p(self._arena_ptr), nbytes, C.c_void_p(self.stream.cuda_stream)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().cg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- running
    def run_hops(self, n_hops: int):
        _check(load().cg_run_hops(self._h, int(n_hops)))

    def run_time(self, t_end: float):
        _check(load().cg_run_time(self._h, float(t_end)))

    def refresh(self):
        _check(load().cg_refresh(self._h))

    def set_TE(self, b: int, T: float, E: float):
        _check(load().cg_set_TE(self._h, b, T, E))

    # -- reading
    def occupation(self, b: int) -> np.ndarray:
        a = np.zeros(self.N[b], np.uint8)
        _check(load().cg_get_occupation(self._h, b, a.ctypes.data_as(C.POINTER(C.c_uint8))))
        return a

    def energies(self, b: int) -> np.ndarray:
        a = np.zeros(self.N[b], np.float64)
        _check(load().cg_get_local_energies(self._h, b, a.ctypes.data_as(C.POINTER(C.c_double))))
        return a

    def phi(self, b: int) -> np.ndarray:
        a = np.zeros(self.N[b], np.float64)
        _check(load().cg_get_phi(self._h, b, a.ctypes.data_as(C.POINTER(C.c_double))))
        return a

    def stats(self, b: int) -> dict:
        s = cg_stats()
        _check(load().cg_get_stats(self._h, b, C.byref(s)))
        d = {k: getattr(s, k) for k, _ in cg_stats._fields_}
        d["phase_cycles"] = list(s.phase_cycles)
        return d

    def clock(self, b: int) -> float:
        t = C.c_double()
        _check(load().cg_get_clock(self._h, b, C.byref(t)))
        return t.value

    def current(self, b: int):
        t, P, sig = C.c_double(), C.c_int64(), C.c_double()
        _check(load().cg_get_current(self._h, b, C.byref(t), C.byref(P), C.byref(sig)))
        return t.value, P.value, sig.value

    def hop_log(self, b: int, cap: int | None = None):
        cap = self.opts.log_hops if cap is None else cap
        lab = np.zeros(max(cap, 1), np.uint64)
        fr = np.zeros(max(cap, 1), np.int32)
        to = np.zeros(max(cap, 1), np.int32)
        cnt = C.c_int64()
        _check(load().cg_get_hop_log(self._h, b, lab.ctypes.data_as(C.POINTER(C.c_uint64)),
                                     fr.ctypes.data_as(C.POINTER(C.c_int32)),
                                     to.ctypes.data_as(C.POINTER(C.c_int32)), cap, C.byref(cnt)))
        k = cnt.value
        return lab[:k].copy(), fr[:k].copy(), to[:k].copy()

    def dos(self, first: int, count: int, e_lo: float, e_hi: float, nbins: int):
        """Density-of-states counts of samples first .. first + count - 1: (occupied[nbins],
        empty[nbins], below, above)."""
        occ = np.zeros(nbins, np.uint64)
        emp = np.zeros(nbins, np.uint64)
        out = np.zeros(2, np.uint64)
        u64 = C.POINTER(C.c_uint64)
        _check(load().cg_dos(self._h, first, count, e_lo, e_hi, nbins, occ.ctypes.data_as(u64),
                             emp.ctypes.data_as(u64), out.ctypes.data_as(u64)))
        return occ, emp, int(out[0]), int(out[1])

    def dos_noalloc(self, first: int, count: int, e_lo: float, e_hi: float, nbins: int):
        """As dos(), through the allocation-free entry point (counts in the library's
        file-scope device array; the output arrays are the caller's)."""
        occ = np.zeros(nbins, np.uint64)
        emp = np.zeros(nbins, np.uint64)
        out = np.zeros(2, np.uint64)
        u64 = C.POINTER(C.c_uint64)
        _check(load().cg_dos_noalloc(self._h, first, count, e_lo, e_hi, nbins, occ.ctypes.data_as(u64),
                                     emp.ctypes.data_as(u64), out.ctypes.data_as(u64)))
        return occ, emp, int(out[0]), int(out[1])

    def save(self, b: int) -> bytes:
        """Checkpoint of sample b (header, state, occupation, energies) as bytes."""
        n = C.c_size_t()
        _check(load().cg_save(self._h, b, None, C.byref(n)))
        buf = (C.c_uint8 * n.value)()
        _check(load().cg_save(self._h, b, C.cast(buf, C.c_void_p), C.byref(n)))
        return bytes(buf[: n.value])

    def load(self, b: int, blob: bytes) -> None:
        """Restore sample b from a checkpoint written by save() for the same sample."""
        buf = (C.c_uint8 * len(blob)).from_buffer_copy(blob)
        _check(load().cg_load(self._h, b, C.cast(buf, C.c_void_p), len(blob)))

    def kernel_time(self):
        """(hop-kernel ms, hop launches, refresh ms, refresh launches) since the last call."""
        hm, hn, rm, rn = C.c_double(), C.c_int64(), C.c_double(), C.c_int64()
        _check(load().cg_take_kernel_time(self._h, C.byref(hm), C.byref(hn), C.byref(rm), C.byref(rn)))
        return hm.value, hn.value, rm.value, rn.value
