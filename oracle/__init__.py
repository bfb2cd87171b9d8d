"""Serial FP64 oracle for the mixed rejection KMC of the 2D lattice Coulomb glass.

TEST INFRASTRUCTURE ONLY.  This package wraps ``liboracle.so`` (plain C, built
from ``oracle.c`` with contraction off).  It may be imported by the test suite,
by the smoke check and by the CPU-baseline leg of the benchmark, never by the
product library, and it shares no code with the GPU path.

The wrapped C functions follow the paper section by section (see the comments in
``oracle.c``): Eq. 1 energy, the single-particle energies, the energy change of a
hop, the mixed algorithm's proposal law (tower sampling over exp(-2r/xi)) and
Metropolis acceptance, step 3b's local-energy update and step 3c's clock.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRC3 = os.path.join(_HERE, "oracle3d.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (the checker's build, not a use of it)."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f)
                                             for f in (_SRC, _SRC3, os.path.join(_HERE, "oracle.h")))
    if force or stale:
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, _SRC3, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("L", C.c_int32), ("n_e", C.c_int32), ("W", C.c_double), ("xi", C.c_double),
                ("rc", C.c_double), ("T", C.c_double), ("E", C.c_double),
                ("seed", C.c_uint64), ("sample_id", C.c_uint32), ("clock_mode", C.c_int32),
                ("pair", C.c_double)]


class _Scalars(C.Structure):
    _fields_ = [("s_last", C.c_uint64), ("s_scan", C.c_uint64), ("hops", C.c_uint64),
                ("P", C.c_int64), ("t", C.c_double), ("H0", C.c_double),
                ("theta_pass", C.c_uint64), ("Gamma", C.c_double), ("Gamma_lab", C.c_double)]


_lib = None


def _bind(path: str):
    """Load a build of the oracle sources and declare the signatures of its functions."""
    L = C.CDLL(path)
    P = C.POINTER
    L.or_philox.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
    L.or_create.argtypes = [P(_Params), P(C.c_void_p)]
    L.or_create.restype = C.c_int
    L.or_create_lazy.argtypes = [P(_Params), P(C.c_void_p)]
    L.or_create_lazy.restype = C.c_int
    L.or_site_eps.argtypes = [C.c_void_p, C.c_int32]
    L.or_site_eps.restype = C.c_double
    L.or_destroy.argtypes = [C.c_void_p]
    L.or_dims.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_int32), P(C.c_int32)]
    L.or_tower.argtypes = [C.c_void_p, P(C.c_uint64), P(C.c_int32), P(C.c_int32),
                           P(C.c_int32), P(C.c_int32), P(C.c_double), P(C.c_double)]
    L.or_draw.argtypes = [C.c_void_p, C.c_uint64, P(C.c_int32), P(C.c_int32), P(C.c_double)]
    L.or_vec_prob.argtypes = [C.c_void_p, C.c_int32]
    L.or_vec_prob.restype = C.c_double
    L.or_invr.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
    L.or_invr.restype = C.c_double
    for f in ("or_get_phi", "or_get_eps"):
        getattr(L, f).argtypes = [C.c_void_p, P(C.c_double)]
    L.or_get_occ.argtypes = [C.c_void_p, P(C.c_uint8)]
    L.or_get_scalars.argtypes = [C.c_void_p, P(_Scalars)]
    L.or_set_occ.argtypes = [C.c_void_p, P(C.c_uint8)]
    L.or_set_occ.restype = C.c_int
    L.or_run.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_int64, P(C.c_uint64),
                         P(C.c_int32), P(C.c_int32), C.c_int64, P(C.c_int64)]
    L.or_run.restype = C.c_int64
    L.or_recompute_eps.argtypes = [C.c_void_p, P(C.c_double)]
    L.or_energy.argtypes = [C.c_void_p]
    L.or_energy.restype = C.c_double
    L.or_move.argtypes = [C.c_void_p, C.c_int32, C.c_int32, P(C.c_double)]
    L.or_move.restype = C.c_double
    L.or_draw_label.argtypes = [C.c_void_p, C.c_uint64, P(C.c_int32), P(C.c_int32), P(C.c_int32),
                                P(C.c_int32), P(C.c_int32), P(C.c_double)]
    L.or_move_pair.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P(C.c_double)]
    L.or_move_pair.restype = C.c_double
    L.or_acceptance.argtypes = [C.c_void_p]
    L.or_acceptance.restype = C.c_double
    L.or_naive_run.argtypes = [C.c_void_p, C.c_double]
    L.or_naive_run.restype = C.c_int64
    L.or3_create.argtypes = [P(_Params), P(C.c_void_p)]
    L.or3_create.restype = C.c_int
    L.or3_destroy.argtypes = [C.c_void_p]
    L.or3_draw.argtypes = [C.c_void_p, C.c_uint64, P(C.c_int32), P(C.c_int32), P(C.c_double)]
    L.or3_invr.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]
    L.or3_invr.restype = C.c_double
    L.or3_run.argtypes = [C.c_void_p, C.c_int64, P(C.c_uint64), P(C.c_int32), P(C.c_int32), C.c_int64]
    L.or3_run.restype = C.c_int64
    L.or3_energy.argtypes = [C.c_void_p]
    L.or3_energy.restype = C.c_double
    L.or3_get.argtypes = [C.c_void_p, P(C.c_uint8), P(C.c_double), P(C.c_double)]
    L.or3_scalars.argtypes = [C.c_void_p, P(_Scalars)]
    L.or3_tower.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_int32), P(C.c_uint64), P(C.c_int32),
                            P(C.c_int32), P(C.c_int32), P(C.c_int32), P(C.c_int32)]
    L.or3_set_occ.argtypes = [C.c_void_p, P(C.c_uint8)]
    L.or_gamma_dt.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64, C.c_double]
    L.or_gamma_dt.restype = C.c_double
    return L


def lib():
    global _lib
    if _lib is None:
        _lib = _bind(build(force=False))
    return _lib


@contextlib.contextmanager
def using_build(path: str):
    """Run the wrappers against another build of the oracle sources (the mutation tests build
    copies with a planted mistake); the regular build is restored on exit."""
    global _lib
    saved = lib()
    _lib = _bind(path)
    try:
        yield
    finally:
        _lib = saved


def build_copy(source_text: str, out_dir: str) -> str:
    """Compile a modified copy of oracle.c (plus oracle3d.c) with the regular flags into
    out_dir; returns the library path."""
    import shutil

    for f in ("oracle.h", "oracle3d.c"):
        shutil.copy(os.path.join(_HERE, f), os.path.join(out_dir, f))
    src = os.path.join(out_dir, "oracle.c")
    with open(src, "w") as fh:
        fh.write(source_text)
    out = os.path.join(out_dir, "liboracle_copy.so")
    subprocess.run(["gcc", *CFLAGS, "-o", out, src, os.path.join(out_dir, "oracle3d.c"), "-lm"], check=True)
    return out


def source() -> str:
    with open(_SRC) as fh:
        return fh.read()


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 of a 4-word counter and 2-word key."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def gamma_dt(seed: int, sample_id: int, hop: int, m: int, Gamma: float) -> float:
    """The exact serial clock's increment for hop `hop` after m proposals (Gamma(m, Gamma))."""
    return lib().or_gamma_dt(seed, sample_id, hop, m, Gamma)


class Oracle:
    """One sample of the serial chain (FP64)."""

    def __init__(self, L, n_e, W=1.0, xi=1.0, rc=6.0, T=0.1, E=0.0, seed=1, sample_id=0,
                 clock_mode=0, lazy=False, pair=0.0):
        """lazy=True: occupation, disorder and proposal law only (no O(N^2) energies; run()
        is unavailable, site_eps() works) -- for lattices too large for the full recompute."""
        self.params = dict(L=L, n_e=n_e, W=W, xi=xi, rc=rc, T=T, E=E, seed=seed,
                           sample_id=sample_id, clock_mode=clock_mode, pair=pair)
        p = _Params(L, n_e, W, xi, rc, T, E, seed, sample_id, clock_mode, pair)
        h = C.c_void_p()
        rc_ = (lib().or_create_lazy if lazy else lib().or_create)(C.byref(p), C.byref(h))
        if rc_ != 0:
            raise ValueError(f"or_create failed ({rc_}) for {self.params}")
        self._h = h
        N, no, nv = C.c_int32(), C.c_int32(), C.c_int32()
        lib().or_dims(h, C.byref(N), C.byref(no), C.byref(nv))
        self.N, self.n_orb, self.n_vec = N.value, no.value, nv.value
        self.L = L

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.or_destroy(h)
            self._h = None

    def tower(self) -> dict:
        thr = np.zeros(self.n_orb, np.uint64)
        size = np.zeros(self.n_orb, np.int32)
        first = np.zeros(self.n_orb, np.int32)
        dx = np.zeros(self.n_vec, np.int32)
        dy = np.zeros(self.n_vec, np.int32)
        ws, G = C.c_double(), C.c_double()
        lib().or_tower(self._h, _ptr(thr, C.c_uint64), _ptr(size, C.c_int32),
                       _ptr(first, C.c_int32), _ptr(dx, C.c_int32), _ptr(dy, C.c_int32),
                       C.byref(ws), C.byref(G))
        return dict(thr=thr, size=size, first=first, dx=dx, dy=dy, wsum=ws.value, Gamma=G.value)

    def draw(self, s: int):
        i, v, u = C.c_int32(), C.c_int32(), C.c_double()
        lib().or_draw(self._h, s, C.byref(i), C.byref(v), C.byref(u))
        return i.value, v.value, u.value

    def vec_prob(self, v: int) -> float:
        return lib().or_vec_prob(self._h, v)

    def invr(self, ddx: int, ddy: int) -> float:
        return lib().or_invr(self._h, ddx, ddy)

    def occ(self) -> np.ndarray:
        a = np.zeros(self.N, np.uint8)
        lib().or_get_occ(self._h, _ptr(a, C.c_uint8))
        return a

    def phi(self) -> np.ndarray:
        a = np.zeros(self.N, np.float64)
        lib().or_get_phi(self._h, _ptr(a, C.c_double))
        return a

    def eps(self) -> np.ndarray:
        a = np.zeros(self.N, np.float64)
        lib().or_get_eps(self._h, _ptr(a, C.c_double))
        return a

    def scalars(self) -> dict:
        s = _Scalars()
        lib().or_get_scalars(self._h, C.byref(s))
        return {k: getattr(s, k) for k, _ in _Scalars._fields_}

    def set_occ(self, n) -> None:
        a = np.ascontiguousarray(n, dtype=np.uint8)
        if lib().or_set_occ(self._h, _ptr(a, C.c_uint8)) != 0:
            raise ValueError("occupation must hold exactly n_e ones")

    def run(self, n_hops: int = 0, t_end: float = -1.0, max_labels: int = 0, log_cap: int | None = None):
        """Advance the chain; returns the log (labels, i, j) of this call's executed hops (a pair
        hop logs two entries with its label).  The default capacity holds every entry."""
        cap = 2 * n_hops if log_cap is None else log_cap
        cap = max(int(cap), 0)
        lab = np.zeros(max(cap, 1), np.uint64)
        li = np.zeros(max(cap, 1), np.int32)
        lj = np.zeros(max(cap, 1), np.int32)
        nlog = C.c_int64()
        done = lib().or_run(self._h, n_hops, t_end, max_labels, _ptr(lab, C.c_uint64),
                            _ptr(li, C.c_int32), _ptr(lj, C.c_int32), cap, C.byref(nlog))
        if done < 0:
            raise ValueError("run() needs the energies: this oracle was created lazy")
        self.last_run_hops = int(done)
        k = min(nlog.value, cap)
        return lab[:k].copy(), li[:k].copy(), lj[:k].copy()

    def draw_label(self, s: int):
        """(is_pair, i, v1, ve, v2, u) of label s (ve = v2 = -1 for a single-hop label)."""
        ip, i, v1, ve, v2, u = (C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(),
                                C.c_double())
        lib().or_draw_label(self._h, s, C.byref(ip), C.byref(i), C.byref(v1), C.byref(ve), C.byref(v2),
                            C.byref(u))
        return ip.value, i.value, v1.value, ve.value, v2.value, u.value

    def move_pair(self, i: int, v1: int, ve: int, v2: int):
        """(acceptance probability, dH) of a pair proposal in the current configuration."""
        dH = C.c_double()
        p = lib().or_move_pair(self._h, i, v1, ve, v2, C.byref(dH))
        return p, dH.value

    def naive_run(self, t_end: float) -> int:
        """Naive serial KMC until the clock reaches t_end; returns the hops executed."""
        done = lib().or_naive_run(self._h, float(t_end))
        if done < 0:
            raise ValueError("naive_run() needs the energies: this oracle was created lazy")
        return int(done)

    def site_eps(self, l: int) -> float:
        """eps_l of the current occupation, O(N), same summation order as the full recompute."""
        return float(lib().or_site_eps(self._h, int(l)))

    def recompute_eps(self) -> np.ndarray:
        a = np.zeros(self.N, np.float64)
        lib().or_recompute_eps(self._h, _ptr(a, C.c_double))
        return a

    def energy(self) -> float:
        return lib().or_energy(self._h)

    def move(self, i: int, v: int):
        dH = C.c_double()
        p = lib().or_move(self._h, i, v, C.byref(dH))
        return p, dH.value

    def acceptance(self) -> float:
        return lib().or_acceptance(self._h)


class Oracle3D:
    """Serial FP64 chain on the simple cubic lattice (L^3 sites), deterministic clock."""

    def __init__(self, L, n_e, W=1.0, xi=1.0, rc=2.0, T=0.1, E=0.0, seed=1, sample_id=0):
        self.params = dict(L=L, n_e=n_e, W=W, xi=xi, rc=rc, T=T, E=E, seed=seed, sample_id=sample_id)
        p = _Params(L, n_e, W, xi, rc, T, E, seed, sample_id, 0, 0.0)
        h = C.c_void_p()
        rc_ = lib().or3_create(C.byref(p), C.byref(h))
        if rc_ != 0:
            raise ValueError(f"or3_create failed ({rc_}) for {self.params}")
        self._h = h
        self.N = L * L * L

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or3_destroy(self._h)
            self._h = None

    def tower(self) -> dict:
        no, nv = C.c_int32(), C.c_int32()
        lib().or3_tower(self._h, C.byref(no), C.byref(nv), None, None, None, None, None, None)
        thr = np.zeros(no.value, np.uint64)
        first = np.zeros(no.value, np.int32)
        size = np.zeros(no.value, np.int32)
        vx, vy, vz = (np.zeros(nv.value, np.int32) for _ in range(3))
        lib().or3_tower(self._h, C.byref(no), C.byref(nv), _ptr(thr, C.c_uint64), _ptr(first, C.c_int32),
                        _ptr(size, C.c_int32), _ptr(vx, C.c_int32), _ptr(vy, C.c_int32), _ptr(vz, C.c_int32))
        return dict(thr=thr, first=first, size=size, dx=vx, dy=vy, dz=vz, Gamma=self.scalars()["Gamma"])

    def draw(self, s: int):
        i, v, u = C.c_int32(), C.c_int32(), C.c_double()
        lib().or3_draw(self._h, s, C.byref(i), C.byref(v), C.byref(u))
        return i.value, v.value, u.value

    def invr(self, dx: int, dy: int, dz: int) -> float:
        return lib().or3_invr(self._h, dx, dy, dz)

    def occ(self) -> np.ndarray:
        a = np.zeros(self.N, np.uint8)
        lib().or3_get(self._h, _ptr(a, C.c_uint8), None, None)
        return a

    def eps(self) -> np.ndarray:
        a = np.zeros(self.N, np.float64)
        lib().or3_get(self._h, None, _ptr(a, C.c_double), None)
        return a

    def phi(self) -> np.ndarray:
        a = np.zeros(self.N, np.float64)
        lib().or3_get(self._h, None, None, _ptr(a, C.c_double))
        return a

    def scalars(self) -> dict:
        s = _Scalars()
        lib().or3_scalars(self._h, C.byref(s))
        return {k: getattr(s, k) for k, _ in _Scalars._fields_}

    def energy(self) -> float:
        return lib().or3_energy(self._h)

    def set_occ(self, n) -> None:
        a = np.ascontiguousarray(n, dtype=np.uint8)
        lib().or3_set_occ(self._h, _ptr(a, C.c_uint8))

    def run(self, n_hops: int):
        lab = np.zeros(max(n_hops, 1), np.uint64)
        li = np.zeros(max(n_hops, 1), np.int32)
        lj = np.zeros(max(n_hops, 1), np.int32)
        k = lib().or3_run(self._h, n_hops, _ptr(lab, C.c_uint64), _ptr(li, C.c_int32), _ptr(lj, C.c_int32), n_hops)
        return lab[:k].copy(), li[:k].copy(), lj[:k].copy()
