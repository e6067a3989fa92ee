"""ctypes binding of the C ABI in include/cc.h (argument marshalling only).

Every entry point forwards torch CUDA/HIP tensors as raw device pointers plus
``torch.cuda.current_stream()``; all arithmetic happens in the HIP kernels.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcc_mi355x.so")

CC_OK, CC_ERR_ARG, CC_ERR_NONFINITE, CC_ERR_DEPTH, CC_ERR_DEVICE, CC_ERR_OOM = 0, -1, -2, -3, -4, -5
CC_FP64, CC_MIXED = 0, 1
CC_ORDER_FAST, CC_ORDER_EXACT = 0, 1
CC_SCREEN_FP64, CC_SCREEN_FP32 = 0, 1
KICK_STATIC_MAX_N = 65536   # CC_KICK_STATIC_MAX_N of include/cc.h

# entry points declared in include/cc.h
SYMBOLS = ("cc_create", "cc_destroy", "cc_set_params", "cc_last_error", "cc_pair_timesteps", "cc_split_labels",
           "cc_kick", "cc_kick_static", "cc_drift", "cc_evolve", "cc_evolve_batch", "cc_diagnostics", "cc_autotune",
           "cc_timing_enable", "cc_timing_report")


class _State(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("x", "y", "z", "vx", "vy", "vz", "m")]


class _Params(C.Structure):
    _fields_ = [("eta", C.c_double), ("eps2", C.c_double), ("G", C.c_double), ("max_depth", C.c_int32),
                ("precision", C.c_int32), ("small_max", C.c_int32), ("kick_order", C.c_int32),
                ("screen", C.c_int32), ("kepler", C.c_int32), ("hold", C.c_int32),
                ("plain", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("tau_pairs", C.c_uint64), ("tau_pairs_alg", C.c_uint64), ("kick_pairs", C.c_uint64),
                ("drifts", C.c_uint64), ("components", C.c_uint64), ("splits", C.c_uint64),
                ("max_depth_seen", C.c_int64), ("t_reached", C.c_double), ("kepler_solves", C.c_uint64)]


class _Tune(C.Structure):
    _fields_ = [("small_max", C.c_int32), ("sweep_split_tiles", C.c_int32), ("kick_groups_per_cu", C.c_int32),
                ("ms_per_step", C.c_double), ("trials", C.c_int32)]


class _KTime(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_uint64), ("ms", C.c_double), ("tau_pairs", C.c_uint64),
                ("kick_pairs", C.c_uint64)]


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libcc_mi355x.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(_LIB_PATH)
    vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    L.cc_create.argtypes = [C.POINTER(vp), i32, C.POINTER(_Params)]
    L.cc_destroy.argtypes = [vp]
    L.cc_destroy.restype = None
    L.cc_set_params.argtypes = [vp, C.POINTER(_Params)]
    L.cc_last_error.argtypes = [vp]
    L.cc_last_error.restype = C.c_char_p
    L.cc_pair_timesteps.argtypes = [vp, C.POINTER(_State), i64, vp, vp, i64, vp, vp]
    L.cc_split_labels.argtypes = [vp, C.POINTER(_State), i64, d, vp, C.POINTER(i64), vp]
    L.cc_kick.argtypes = [vp, C.POINTER(_State), i64, vp, d, vp]
    L.cc_kick_static.argtypes = [vp, C.POINTER(_State), i64, vp, d, vp]
    L.cc_drift.argtypes = [vp, C.POINTER(_State), i64, vp, d, vp]
    L.cc_evolve.argtypes = [vp, C.POINTER(_State), i64, d, d, C.POINTER(_Stats), vp]
    L.cc_evolve_batch.argtypes = [vp, C.POINTER(_State), C.POINTER(i64), i32, d, d, C.POINTER(_Stats), vp]
    L.cc_diagnostics.argtypes = [vp, C.POINTER(_State), i64, C.POINTER(d), vp]
    L.cc_autotune.argtypes = [vp, C.POINTER(_State), i64, d, C.POINTER(_Tune), vp]
    L.cc_timing_enable.argtypes = [vp, i32]
    L.cc_timing_report.argtypes = [vp, C.POINTER(_KTime), i32]
    for f in SYMBOLS:
        if f not in ("cc_destroy", "cc_last_error"):
            getattr(L, f).restype = C.c_int
    _lib = L
    return L


class CCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cc error {code}: {msg}")
        self.code = code


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


@dataclass
class State:
    """SoA FP64 particle state on the GPU (contiguous torch tensors)."""
    x: torch.Tensor
    y: torch.Tensor
    z: torch.Tensor
    vx: torch.Tensor
    vy: torch.Tensor
    vz: torch.Tensor
    m: torch.Tensor

    FIELDS = ("x", "y", "z", "vx", "vy", "vz", "m")

    @property
    def n(self) -> int:
        return int(self.m.shape[0])

    @classmethod
    def from_numpy(cls, p, device="cuda") -> "State":
        """From any object with float64 numpy attributes x..m (e.g. synth.Particles)."""
        return cls(*(torch.from_numpy(np.ascontiguousarray(getattr(p, f), dtype=np.float64)).to(device)
                     for f in cls.FIELDS))

    def to_numpy(self):
        return {f: getattr(self, f).detach().cpu().numpy() for f in self.FIELDS}

    def copy(self) -> "State":
        return State(*(getattr(self, f).clone() for f in self.FIELDS))

    def _c(self) -> _State:
        for f in self.FIELDS:
            t = getattr(self, f)
            if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
                raise TypeError(f"state.{f} must be a contiguous float64 GPU tensor")
            if t.shape[0] != self.n:
                raise ValueError("state arrays differ in length")
        return _State(*(t.data_ptr() for t in (getattr(self, f) for f in self.FIELDS)))


def _stats(st: _Stats) -> dict:
    return {k: getattr(st, k) for k, _ in _Stats._fields_}


class Context:
    """One library context (device scratch memory, parameters)."""

    def __init__(self, device: int = 0, eta: float = 0.01, eps2: float = 0.0, G: float = 1.0,
                 max_depth: int = 48, precision: int = CC_FP64, small_max: int = 0,
                 kick_order: int = CC_ORDER_FAST, screen: int = CC_SCREEN_FP64, kepler: int = 0,
                 hold: int = 0, plain: int = 0):
        self._L = load_library()
        self._p = _Params(eta, eps2, G, max_depth, precision, small_max, kick_order, screen, kepler, hold, plain)
        h = C.c_void_p()
        rc = self._L.cc_create(C.byref(h), device, C.byref(self._p))
        if rc != CC_OK:
            raise CCError(rc, "cc_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._L.cc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != CC_OK:
            raise CCError(rc, self._L.cc_last_error(self._h).decode())

    def set_params(self, **kw):
        for k, v in kw.items():
            setattr(self._p, k, v)
        self._check(self._L.cc_set_params(self._h, C.byref(self._p)))

    @property
    def params(self) -> dict:
        return {k: getattr(self._p, k) for k, _ in _Params._fields_}

    def pair_timesteps(self, s: State, pi: torch.Tensor, pj: torch.Tensor) -> torch.Tensor:
        pi = pi.to(device=s.m.device, dtype=torch.int32).contiguous()
        pj = pj.to(device=s.m.device, dtype=torch.int32).contiguous()
        out = torch.empty(pi.shape[0], dtype=torch.float64, device=s.m.device)
        self._check(self._L.cc_pair_timesteps(self._h, C.byref(s._c()), s.n, _ptr(pi), _ptr(pj), pi.shape[0],
                                              _ptr(out), _stream()))
        return out

    def split_labels(self, s: State, h: float, count: bool = True):
        lab = torch.empty(s.n, dtype=torch.int32, device=s.m.device)
        nt = C.c_int64(-1)
        self._check(self._L.cc_split_labels(self._h, C.byref(s._c()), s.n, h, _ptr(lab),
                                            C.byref(nt) if count else None, _stream()))
        return lab, (int(nt.value) if count else None)

    def kick(self, s: State, h: float, label: torch.Tensor | None = None):
        if label is not None:
            label = label.to(device=s.m.device, dtype=torch.int32).contiguous()
        self._check(self._L.cc_kick(self._h, C.byref(s._c()), s.n, _ptr(label), h, _stream()))

    def kick_static(self, s: State, h: float, label: torch.Tensor | None = None):
        """cc_kick without any allocation (scratch in a static device array;
        n <= KICK_STATIC_MAX_N)."""
        if label is not None:
            label = label.to(device=s.m.device, dtype=torch.int32).contiguous()
        self._check(self._L.cc_kick_static(self._h, C.byref(s._c()), s.n, _ptr(label), h, _stream()))

    def drift(self, s: State, h: float, mask: torch.Tensor | None = None):
        if mask is not None:
            mask = mask.to(device=s.m.device, dtype=torch.uint8).contiguous()
        self._check(self._L.cc_drift(self._h, C.byref(s._c()), s.n, _ptr(mask), h, _stream()))

    def evolve(self, s: State, dt: float, t_end: float, raise_on_error: bool = True):
        st = _Stats()
        rc = self._L.cc_evolve(self._h, C.byref(s._c()), s.n, dt, t_end, C.byref(st), _stream())
        if raise_on_error:
            self._check(rc)
        return (_stats(st) if raise_on_error else (rc, _stats(st)))

    def evolve_batch(self, s: State, offsets, dt: float, t_end: float, raise_on_error: bool = True):
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        ncl = off.shape[0] - 1
        st = (_Stats * ncl)()
        rc = self._L.cc_evolve_batch(self._h, C.byref(s._c()), off.ctypes.data_as(C.POINTER(C.c_int64)), ncl, dt,
                                     t_end, st, _stream())
        if raise_on_error:
            self._check(rc)
            return [_stats(st[c]) for c in range(ncl)]
        return rc, [_stats(st[c]) for c in range(ncl)]

    def diagnostics(self, s: State) -> dict:
        out = (C.c_double * 12)()
        self._check(self._L.cc_diagnostics(self._h, C.byref(s._c()), s.n, out, _stream()))
        o = np.array(out[:])
        return dict(ekin=o[0], epot=o[1], energy=o[0] + o[1], P=o[2:5], L=o[5:8], com=o[8:11], mass=o[11])

    def autotune(self, s: State, dt: float) -> dict:
        """Time one global step of s (read only) per launch-shape candidate and
        keep the fastest in this context; returns the choice."""
        t = _Tune()
        self._check(self._L.cc_autotune(self._h, C.byref(s._c()), s.n, dt, C.byref(t), _stream()))
        self._p.small_max = t.small_max
        return dict(small_max=t.small_max, sweep_split_tiles=t.sweep_split_tiles,
                    kick_groups_per_cu=t.kick_groups_per_cu, ms_per_step=t.ms_per_step, trials=t.trials)

    def timing(self, enable: bool):
        self._check(self._L.cc_timing_enable(self._h, 1 if enable else 0))

    def timing_report(self) -> dict:
        recs = (_KTime * 32)()
        k = self._L.cc_timing_report(self._h, recs, 32)
        if k < 0:
            self._check(k)
        return {recs[i].name.decode(): dict(launches=recs[i].launches, ms=recs[i].ms, tau_pairs=recs[i].tau_pairs,
                                            kick_pairs=recs[i].kick_pairs) for i in range(min(k, 32))}
