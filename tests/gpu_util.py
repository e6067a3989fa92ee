"""Helpers shared by the GPU tests (inputs and comparisons; no arithmetic of the method)."""
import numpy as np

FIELDS = ("x", "y", "z", "vx", "vy", "vz")


def assert_state_equal(got: dict, ref, what=""):
    for f in FIELDS:
        a, b = got[f], getattr(ref, f)
        if not np.array_equal(a, b):
            bad = np.flatnonzero(a != b)
            d = np.max(np.abs(a - b))
            raise AssertionError(f"{what} {f}: {bad.size} entries differ (first {bad[:5]}, max |diff| {d:.3e})")
