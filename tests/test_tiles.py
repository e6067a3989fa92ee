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


def _blocked(shim, T, t0, count):
    out = np.zeros(2 * count, np.int32)
    shim.blocked_tiles(C.c_int(T), C.c_int64(t0), C.c_int64(count), out.ctypes.data_as(C.POINTER(C.c_int32)))
    return out[0::2].astype(np.int64), out[1::2].astype(np.int64)


@pytest.mark.parametrize("T", [1, 5, 31, 64, 255, 511, 512, 513, 527, 528, 529, 1000, 4096, 4097])
def test_blocked_tile_is_a_permutation_of_the_triangle(shim, T):
    """Every tile of the upper triangle exactly once; below 512 tiles per
    side the order is the row-by-row one."""
    tot = T * (T + 1) // 2
    ti, tj = _blocked(shim, T, 0, tot)
    assert np.all((0 <= ti) & (ti <= tj) & (tj < T))
    assert np.unique(ti * T + tj).size == tot
    if T < 512:
        want_i, want_j = np.triu_indices(T)
        assert np.array_equal(ti, want_i) and np.array_equal(tj, want_j)


@pytest.mark.parametrize("T", [512, 1000, 4096])
def test_blocked_tile_keeps_runs_inside_super_tiles(shim, T):
    """Consecutive runs of 256 tiles (one XCD's share of a launch, in order)
    lie in at most three super-tiles: under 6 x 16 tile rows and columns in
    all; the row-by-row order of a 4096-tile grid touches 257 per run."""
    tot = T * (T + 1) // 2
    ti, tj = _blocked(shim, T, 0, tot)
    worst = 0
    for a in range(0, tot - 256, 256):
        rows = np.unique(ti[a:a + 256]).size
        cols = np.unique(tj[a:a + 256]).size
        worst = max(worst, rows + cols)
    assert worst < 6 * 16, worst
