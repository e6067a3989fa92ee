"""The FP32 edge screen of the mixed path (host build of the device header,
with the hardware reciprocal and square root stood in for by correctly
rounded ones pushed by up to two units in the last place) against the
oracle's literal FP64 edge test tau(i,j) < h (eqs. 19-20).

Whenever the screen decides, its decision must equal the literal one; it may
only answer UNSURE.  The pairs and thresholds are those of the FP64 screen's
test: separations, speeds, mass ratios and approach angles over many decades,
thresholds at each pair's own tau, within a few ulps and a few hundred ulps of
it, and at random."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle

from .test_screen64 import _pairs_state

HERE = os.path.dirname(os.path.abspath(__file__))
NO, EDGE, UNSURE = 0, 1, 2


def _build(tmp_path_factory, name, defines=()):
    out = str(tmp_path_factory.mktemp(name) / f"lib{name}.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    *defines, os.path.join(HERE, "screen32_shim.cpp"), "-o", out], check=True)
    return C.CDLL(out)


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    return _build(tmp_path_factory, "screen32")


@pytest.fixture(scope="module")
def shim_cut(tmp_path_factory):
    """Planted mistake: terms decided at face value (no slack for the error
    bound)."""
    return _build(tmp_path_factory, "screen32cut", ["-DCC_SCREEN32_SLACK=0.0f"])


def _decide(shim, s, pi, pj, h, eta, eps2, G):
    d = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    pi = np.ascontiguousarray(pi, np.int32)
    pj = np.ascontiguousarray(pj, np.int32)
    h = np.ascontiguousarray(h, np.float64)
    out = np.zeros(len(pi), np.int32)
    shim.screen32_pairs(d(s.x), d(s.y), d(s.z), d(s.vx), d(s.vy), d(s.vz), d(s.m),
                        pi.ctypes.data_as(C.POINTER(C.c_int32)), pj.ctypes.data_as(C.POINTER(C.c_int32)),
                        C.c_int64(len(pi)), d(h), C.c_double(eta), C.c_double(eps2), C.c_double(G),
                        out.ctypes.data_as(C.POINTER(C.c_int32)))
    return out


def _cases(rng, tau, n):
    k = rng.integers(-400, 401, n).astype(np.float64)
    k[: n // 4] = rng.integers(-3, 4, n // 4)
    return {
        "near": tau * (1.0 + k * 2.0 ** -52),
        "exact": tau.copy(),
        "up": np.nextafter(tau, np.inf),
        "down": np.nextafter(tau, 0.0),
        "near32": tau * (1.0 + rng.integers(-400, 401, n) * 2.0 ** -23),
        "random": tau * 10.0 ** rng.uniform(-3, 3, n),
    }


@pytest.mark.parametrize("eta,eps2,G", [(0.01, 0.0, 1.0), (0.3, 0.0, 1.0), (1.0, 1e-8, 4.3e-3),
                                         (0.003, 0.0, 1.0)])
def test_fp32_screen_never_contradicts_literal_test(shim, eta, eps2, G):
    rng = np.random.default_rng(3205 + int(eta * 1000))
    n = 40000
    s, pi, pj = _pairs_state(rng, n)
    p = oracle.Params(eta=eta, eps2=eps2, G=G)
    tau = oracle.pair_timesteps(s, pi, pj, p)
    ok = tau > 0
    for name, h in _cases(rng, tau, n).items():
        sel = ok & (h > 0) & np.isfinite(h)
        dec = _decide(shim, s, pi[sel], pj[sel], h[sel], eta, eps2, G)
        ref = tau[sel] < h[sel]
        decided = dec != UNSURE
        bad = decided & ((dec == EDGE) != ref)
        assert not bad.any(), f"{name}: {bad.sum()} wrong decisions, first at pair {np.flatnonzero(bad)[:5]}"
        if name == "random":
            # far from the threshold the FP32 screen decides most pairs in its range
            assert decided.mean() > 0.5, decided.mean()
        if name in ("exact", "up", "down"):
            # within an ulp or two of tau the FP32 screen cannot decide
            assert decided.mean() < 0.01, (name, decided.mean())


def test_fp32_screen_with_no_slack_is_caught(shim_cut):
    """The same cases find the planted mistake: near-threshold pairs decided
    wrongly once the error bound is not allowed for."""
    rng = np.random.default_rng(11)
    n = 40000
    s, pi, pj = _pairs_state(rng, n)
    p = oracle.Params(eta=0.01)
    tau = oracle.pair_timesteps(s, pi, pj, p)
    ok = tau > 0
    wrong = 0
    for name, h in _cases(rng, tau, n).items():
        sel = ok & (h > 0) & np.isfinite(h)
        dec = _decide(shim_cut, s, pi[sel], pj[sel], h[sel], 0.01, 0.0, 1.0)
        wrong += int(((dec != UNSURE) & ((dec == EDGE) != (tau[sel] < h[sel]))).sum())
    assert wrong > 0
