"""MI355X (gfx950) implementation of the connected-component Hamiltonian-
splitting N-body integrator (Janes, Pelupessy & Portegies Zwart, arXiv:1407.7105).

The compute path is the HIP library ``libcc_mi355x.so`` (C ABI in
``include/cc.h``); this package is a thin ctypes binding that passes torch
device pointers and the current HIP stream.  There is no CPU fallback: if the
library is missing, importing :mod:`paper_1407_7105_amd.cc` raises.
"""
from .cc import (CC_FP64, CC_MIXED, CC_ORDER_EXACT, CC_ORDER_FAST, CC_SCREEN_FP32, CC_SCREEN_FP64,  # noqa: F401
                 CCError, Context, State, lib_path, load_library)

__all__ = ["Context", "State", "CCError", "CC_FP64", "CC_MIXED", "CC_ORDER_FAST", "CC_ORDER_EXACT", "CC_SCREEN_FP64",
           "CC_SCREEN_FP32", "lib_path", "load_library"]
