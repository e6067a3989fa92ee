"""ctypes wrapper of the FP64 CPU oracle (``oracle/cc_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain CPU reference that the GPU
library is checked against.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this module; the GPU
library never calls it and has no fallback to it.

State arguments are any object with float64 numpy attributes
x, y, z, vx, vy, vz, m (for instance ``synth.Particles``); the arrays are
updated in place by the integrator entry points.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cc_oracle.c")
_LIB = os.path.join(_HERE, "libcc_oracle.so")

CCO_OK, CCO_ERR_ARG, CCO_ERR_NONFINITE, CCO_ERR_DEPTH, CCO_ERR_OOM = 0, -1, -2, -3, -5

# Flags: every operation a single IEEE binary64 operation (no contraction,
# no fast-math, no host-specific vector ISA).
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/libcc_oracle.so."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _State(C.Structure):
    _fields_ = [(k, C.POINTER(C.c_double)) for k in ("x", "y", "z", "vx", "vy", "vz", "m")]


class _Params(C.Structure):
    _fields_ = [("eta", C.c_double), ("eps2", C.c_double), ("G", C.c_double), ("max_depth", C.c_int),
                ("kepler", C.c_int), ("hold", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("tau_evals", C.c_uint64), ("kick_pairs", C.c_uint64), ("drifts", C.c_uint64),
                ("components", C.c_uint64), ("splits", C.c_uint64), ("max_depth_seen", C.c_int64),
                ("t_reached", C.c_double), ("kepler_solves", C.c_uint64)]


@dataclass
class Params:
    eta: float = 0.01
    eps2: float = 0.0
    G: float = 1.0
    max_depth: int = 48
    kepler: int = 0      # 1: CC_KEPLER (two-particle components by the Kepler solution)
    hold: int = 0        # 1: the HOLD split (fast particles recursed into as one set)

    def c(self) -> _Params:
        return _Params(self.eta, self.eps2, self.G, self.max_depth, self.kepler, self.hold)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P, S = C.POINTER(_Params), C.POINTER(_State)
        i64p, u64p, i32p, dp, u8p = (C.POINTER(C.c_int64), C.POINTER(C.c_uint64),
                                     C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_uint8))
        L.cco_tau.restype = C.c_double
        L.cco_tau.argtypes = [P, S, C.c_int64, C.c_int64]
        L.cco_tau_parts.restype = None
        L.cco_tau_parts.argtypes = [P, S, C.c_int64, C.c_int64, dp]
        L.cco_pair_timesteps.argtypes = [P, S, C.c_int64, i32p, i32p, C.c_int64, dp]
        L.cco_split_bfs.argtypes = [P, S, i64p, C.c_int64, C.c_double, i64p, u64p]
        L.cco_split_uf.argtypes = [P, S, i64p, C.c_int64, C.c_double, i64p]
        L.cco_split_labels.argtypes = [P, S, C.c_int64, C.c_double, i32p, i64p, u64p]
        L.cco_kick.argtypes = [P, S, i64p, C.c_int64, i64p, C.c_double, u64p]
        L.cco_drift.argtypes = [S, i64p, C.c_int64, u8p, C.c_double]
        L.cco_evolve.argtypes = [P, S, C.c_int64, C.c_double, C.c_double, C.POINTER(_Stats)]
        L.cco_evolve_batch.argtypes = [P, S, i64p, C.c_int32, C.c_double, C.c_double, C.POINTER(_Stats)]
        L.cco_accel.argtypes = [P, S, C.c_int64, i64p, C.c_int64, dp, dp, dp]
        L.cco_accel_compensated.argtypes = [P, S, C.c_int64, i64p, C.c_int64, dp, dp, dp]
        L.cco_diagnostics.argtypes = [P, S, C.c_int64, dp]
        L.cco_kepler.argtypes = [C.c_double, dp, C.c_double]
        for f in ("cco_pair_timesteps", "cco_split_bfs", "cco_split_uf", "cco_split_labels", "cco_kick",
                  "cco_drift", "cco_evolve", "cco_evolve_batch", "cco_accel", "cco_accel_compensated",
                  "cco_diagnostics", "cco_kepler"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct=C.c_double):
    return a.ctypes.data_as(C.POINTER(ct))


def _check(s):
    for k in ("x", "y", "z", "vx", "vy", "vz", "m"):
        a = getattr(s, k)
        if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous):
            raise TypeError(f"state.{k} must be a contiguous float64 numpy array")


def _state(s) -> _State:
    _check(s)
    return _State(*(_ptr(getattr(s, k)) for k in ("x", "y", "z", "vx", "vy", "vz", "m")))


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed with code {code}")
        self.code = code


def _rc(code: int, what: str):
    if code != CCO_OK:
        raise OracleError(code, what)


def _params(p) -> _Params:
    return (p or Params()).c()


def tau(s, i: int, j: int, p: Params | None = None) -> float:
    return lib().cco_tau(C.byref(_params(p)), C.byref(_state(s)), i, j)


def tau_parts(s, i: int, j: int, p: Params | None = None) -> np.ndarray:
    out = np.zeros(5)
    lib().cco_tau_parts(C.byref(_params(p)), C.byref(_state(s)), i, j, _ptr(out))
    return out


def pair_timesteps(s, pi: np.ndarray, pj: np.ndarray, p: Params | None = None) -> np.ndarray:
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    pj = np.ascontiguousarray(pj, dtype=np.int32)
    out = np.zeros(pi.shape[0])
    _rc(lib().cco_pair_timesteps(C.byref(_params(p)), C.byref(_state(s)), len(s.m), _ptr(pi, C.c_int32),
                                 _ptr(pj, C.c_int32), pi.shape[0], _ptr(out)), "cco_pair_timesteps")
    return out


def split_bfs(s, h: float, I: np.ndarray | None = None, p: Params | None = None):
    """Returns (labels per element of I, tau evaluations)."""
    I = np.arange(len(s.m), dtype=np.int64) if I is None else np.ascontiguousarray(I, dtype=np.int64)
    lab = np.zeros(I.shape[0], np.int64)
    ev = C.c_uint64(0)
    _rc(lib().cco_split_bfs(C.byref(_params(p)), C.byref(_state(s)), _ptr(I, C.c_int64), I.shape[0], h,
                            _ptr(lab, C.c_int64), C.byref(ev)), "cco_split_bfs")
    return lab, int(ev.value)


def split_uf(s, h: float, I: np.ndarray | None = None, p: Params | None = None) -> np.ndarray:
    I = np.arange(len(s.m), dtype=np.int64) if I is None else np.ascontiguousarray(I, dtype=np.int64)
    lab = np.zeros(I.shape[0], np.int64)
    _rc(lib().cco_split_uf(C.byref(_params(p)), C.byref(_state(s)), _ptr(I, C.c_int64), I.shape[0], h,
                           _ptr(lab, C.c_int64)), "cco_split_uf")
    return lab


def split_labels(s, h: float, p: Params | None = None):
    """Labels (int32, smallest index of the component) for all particles,
    number of non-trivial components, tau evaluations."""
    n = len(s.m)
    lab = np.zeros(n, np.int32)
    nt = C.c_int64(0)
    ev = C.c_uint64(0)
    _rc(lib().cco_split_labels(C.byref(_params(p)), C.byref(_state(s)), n, h, _ptr(lab, C.c_int32),
                               C.byref(nt), C.byref(ev)), "cco_split_labels")
    return lab, int(nt.value), int(ev.value)


def kick(s, h: float, label: np.ndarray | None = None, I: np.ndarray | None = None,
         p: Params | None = None) -> int:
    I = np.arange(len(s.m), dtype=np.int64) if I is None else np.ascontiguousarray(I, dtype=np.int64)
    lp = None
    if label is not None:
        label = np.ascontiguousarray(label, dtype=np.int64)
        lp = _ptr(label, C.c_int64)
    pairs = C.c_uint64(0)
    _rc(lib().cco_kick(C.byref(_params(p)), C.byref(_state(s)), _ptr(I, C.c_int64), I.shape[0], lp, h,
                       C.byref(pairs)), "cco_kick")
    return int(pairs.value)


def drift(s, h: float, mask: np.ndarray | None = None, I: np.ndarray | None = None):
    I = np.arange(len(s.m), dtype=np.int64) if I is None else np.ascontiguousarray(I, dtype=np.int64)
    mp = None
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        mp = _ptr(mask, C.c_uint8)
    _rc(lib().cco_drift(C.byref(_state(s)), _ptr(I, C.c_int64), I.shape[0], mp, h), "cco_drift")


def _stats_dict(st: _Stats) -> dict:
    return {k: getattr(st, k) for k, _ in _Stats._fields_}


def evolve(s, dt: float, t_end: float, p: Params | None = None, raise_on_error: bool = True):
    """Integrate in place; returns (return code, stats dict)."""
    st = _Stats()
    rc = lib().cco_evolve(C.byref(_params(p)), C.byref(_state(s)), len(s.m), dt, t_end, C.byref(st))
    if raise_on_error:
        _rc(rc, "cco_evolve")
    return rc, _stats_dict(st)


def evolve_batch(s, offsets: np.ndarray, dt: float, t_end: float, p: Params | None = None,
                 raise_on_error: bool = True):
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    ncl = off.shape[0] - 1
    st = (_Stats * ncl)()
    rc = lib().cco_evolve_batch(C.byref(_params(p)), C.byref(_state(s)), _ptr(off, C.c_int64), ncl, dt,
                                t_end, st)
    if raise_on_error:
        _rc(rc, "cco_evolve_batch")
    return rc, [_stats_dict(st[c]) for c in range(ncl)]


def accel(s, idx: np.ndarray | None = None, p: Params | None = None, compensated: bool = False):
    n = len(s.m)
    idx = np.arange(n, dtype=np.int64) if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
    ax, ay, az = (np.zeros(idx.shape[0]) for _ in range(3))
    f = lib().cco_accel_compensated if compensated else lib().cco_accel
    _rc(f(C.byref(_params(p)), C.byref(_state(s)), n, _ptr(idx, C.c_int64), idx.shape[0], _ptr(ax),
          _ptr(ay), _ptr(az)), "cco_accel")
    return np.stack([ax, ay, az], axis=1)


def kepler(mu: float, r, v, dt: float):
    """The oracle's two-body flow: relative position r and velocity v (3-vectors)
    advanced by dt under mu = G (m_i + m_j).  Returns (r, v)."""
    rv = np.ascontiguousarray(np.concatenate([np.asarray(r, float), np.asarray(v, float)]), dtype=np.float64)
    _rc(lib().cco_kepler(mu, _ptr(rv), dt), "cco_kepler")
    return rv[:3].copy(), rv[3:].copy()


def diagnostics(s, p: Params | None = None) -> dict:
    out = np.zeros(12)
    _rc(lib().cco_diagnostics(C.byref(_params(p)), C.byref(_state(s)), len(s.m), _ptr(out)),
        "cco_diagnostics")
    return dict(ekin=out[0], epot=out[1], energy=out[0] + out[1], P=out[2:5].copy(), L=out[5:8].copy(),
                com=out[8:11].copy(), mass=out[11])
