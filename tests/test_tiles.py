"""The sweep's tile numbering (host build of the device header): tile t of the
upper triangle of a T x T grid, numbered row by row, against an explicit
enumeration of the triangle; every tile once, rows and columns in range."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("tiles") / "libtiles.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    os.path.join(HERE, "tiles_shim.cpp"), "-o", out], check=True)
    return C.CDLL(out)


def _tiles(shim, T, t0, count):
    out = np.zeros(2 * count, np.int32)
    shim.tri_tiles(C.c_int(T), C.c_int64(t0), C.c_int64(count), out.ctypes.data_as(C.POINTER(C.c_int32)))
    return out[0::2], out[1::2]


@pytest.mark.parametrize("T", [1, 2, 3, 5, 63, 64, 65, 256, 1000, 4097])
def test_tri_tile_enumerates_the_triangle(shim, T):
    tot = T * (T + 1) // 2
    ti, tj = _tiles(shim, T, 0, tot)
    want_i, want_j = np.triu_indices(T)           # row by row, tj >= ti
    assert np.array_equal(ti, want_i) and np.array_equal(tj, want_j)


@pytest.mark.parametrize("T", [4096, 16384, 65535])
def test_tri_tile_large_grids_at_row_boundaries(shim, T):
    # the first and last tile of sampled rows, where the rounded root matters
    rows = np.unique(np.concatenate([np.arange(0, 50), np.linspace(0, T - 1, 400).astype(np.int64),
                                     np.arange(T - 50, T)]))
    for r in rows:
        first = int(r) * T - int(r) * (int(r) - 1) // 2
        ti, tj = _tiles(shim, T, first, T - int(r))
        assert np.all(ti == r) and np.array_equal(tj, np.arange(r, T)), r
