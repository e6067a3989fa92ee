"""The certified FP64 edge screen (host build of the device header) against the
oracle's literal edge test tau(i,j) < h (eqs. 19-20).

Whenever the screen decides (EDGE or NO) its decision must equal the literal
FP64 one; it may only answer UNSURE.  Thresholds are placed within a few
hundred ulps of each pair's own tau, where a wrong margin would show, and at
random, where the screen should almost always decide.
"""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle
from synth import Particles

HERE = os.path.dirname(os.path.abspath(__file__))
NO, EDGE, UNSURE = 0, 1, 2


def _build_shim(tmp_path_factory, name, defines=()):
    out = str(tmp_path_factory.mktemp(name) / f"lib{name}.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    *defines, os.path.join(HERE, "screen64_shim.cpp"), "-o", out], check=True)
    return C.CDLL(out)


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    return _build_shim(tmp_path_factory, "screen64")


@pytest.fixture(scope="module")
def shim_cut(tmp_path_factory):
    """The same header with the far-pair margin cut to one half (a planted
    mistake: the bound then only guarantees tau >= h/2)."""
    return _build_shim(tmp_path_factory, "screen64cut", ["-DCC_FAR64_MARGIN=0.5"])


def _decide(shim, s, pi, pj, h, eta, eps2, G):
    d = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    pi = np.ascontiguousarray(pi, np.int32)
    pj = np.ascontiguousarray(pj, np.int32)
    h = np.ascontiguousarray(h, np.float64)
    out = np.zeros(len(pi), np.int32)
    shim.screen64_pairs(d(s.x), d(s.y), d(s.z), d(s.vx), d(s.vy), d(s.vz), d(s.m),
                        pi.ctypes.data_as(C.POINTER(C.c_int32)), pj.ctypes.data_as(C.POINTER(C.c_int32)),
                        C.c_int64(len(pi)), d(h), C.c_double(eta), C.c_double(eps2), C.c_double(G),
                        out.ctypes.data_as(C.POINTER(C.c_int32)))
    return out


# the far-pair test as the on-chip split calls it (far64), and in the sweep's
# form (far64b: box check, fused multiply-adds, mu from the two G m)
FAR_FORMS = ["far64_pairs", "far64b_pairs"]


def _far(shim, s, pi, pj, h, eta, eps2, G, form="far64_pairs"):
    d = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    pi = np.ascontiguousarray(pi, np.int32)
    pj = np.ascontiguousarray(pj, np.int32)
    h = np.ascontiguousarray(h, np.float64)
    out = np.zeros(len(pi), np.int32)
    getattr(shim, form)(d(s.x), d(s.y), d(s.z), d(s.vx), d(s.vy), d(s.vz), d(s.m),
                     pi.ctypes.data_as(C.POINTER(C.c_int32)), pj.ctypes.data_as(C.POINTER(C.c_int32)),
                     C.c_int64(len(pi)), d(h), C.c_double(eta), C.c_double(eps2), C.c_double(G),
                     out.ctypes.data_as(C.POINTER(C.c_int32)))
    return out.astype(bool)


def _pairs_state(rng, n):
    """n independent pairs (2n particles) spanning separations, speeds, mass
    ratios and approach angles far wider than a star cluster's."""
    def unit(k):
        v = rng.normal(size=(k, 3))
        return v / np.linalg.norm(v, axis=1)[:, None]
    r = 10.0 ** rng.uniform(-7, 2, n)
    u = 10.0 ** rng.uniform(-7, 3, n)
    cosang = rng.uniform(-1, 1, n)
    cosang[: n // 8] = -1.0          # head-on approach: t' large, denominators near or below zero
    cosang[n // 8: n // 4] = 0.0     # circular-like: q.u = 0
    qd = unit(n)
    # velocity with the chosen angle to q
    perp = unit(n)
    perp -= (perp * qd).sum(1)[:, None] * qd
    perp /= np.linalg.norm(perp, axis=1)[:, None]
    sinang = np.sqrt(np.maximum(0.0, 1 - cosang ** 2))
    ud = cosang[:, None] * qd + sinang[:, None] * perp
    base = rng.uniform(-1, 1, (n, 3))
    vb = rng.uniform(-1, 1, (n, 3))
    x = np.empty((2 * n, 3))
    v = np.empty((2 * n, 3))
    x[0::2] = base + r[:, None] * qd
    x[1::2] = base
    v[0::2] = vb + u[:, None] * ud
    v[1::2] = vb
    v[2 * (n // 16): 2 * (n // 16) + 2: 2] = v[2 * (n // 16) + 1: 2 * (n // 16) + 3: 2]  # a zero |u| pair
    m = 10.0 ** rng.uniform(-9, 0, 2 * n)
    s = Particles(x=x[:, 0].copy(), y=x[:, 1].copy(), z=x[:, 2].copy(), vx=v[:, 0].copy(),
                  vy=v[:, 1].copy(), vz=v[:, 2].copy(), m=m)
    pi = np.arange(0, 2 * n, 2, dtype=np.int32)
    pj = pi + 1
    return s, pi, pj


@pytest.mark.parametrize("eta,eps2,G", [(0.01, 0.0, 1.0), (0.3, 0.0, 1.0), (1.0, 1e-8, 4.3e-3),
                                         (0.003, 0.0, 1.0)])
def test_screen_never_contradicts_literal_test(shim, eta, eps2, G):
    rng = np.random.default_rng(7105 + int(eta * 1000))
    n = 40000
    s, pi, pj = _pairs_state(rng, n)
    p = oracle.Params(eta=eta, eps2=eps2, G=G)
    tau = oracle.pair_timesteps(s, pi, pj, p)
    assert np.all(np.isfinite(tau)) and np.all(tau >= 0)
    ok = tau > 0
    # thresholds at the pair's own tau, +- a few ulps, +- a few hundred ulps, and at random
    k = rng.integers(-400, 401, n).astype(np.float64)
    k[: n // 4] = rng.integers(-3, 4, n // 4)
    cases = {
        "near": tau * (1.0 + k * 2.0 ** -52),
        "exact": tau.copy(),
        "up": np.nextafter(tau, np.inf),
        "down": np.nextafter(tau, 0.0),
        "random": tau * 10.0 ** rng.uniform(-3, 3, n),
    }
    for name, h in cases.items():
        sel = ok & (h > 0) & np.isfinite(h)
        dec = _decide(shim, s, pi[sel], pj[sel], h[sel], eta, eps2, G)
        ref = tau[sel] < h[sel]
        decided = dec != UNSURE
        bad = decided & ((dec == EDGE) != ref)
        assert not bad.any(), f"{name}: {bad.sum()} wrong decisions, first at pair {np.flatnonzero(bad)[:5]}"
        if name == "random":
            # far from the threshold, and with h inside the screen's certified
            # range, the screen decides essentially everything
            inr = (h[sel] >= 2.0 ** -60) & (h[sel] <= 2.0 ** 60)
            assert inr.mean() > 0.99 and decided[inr].mean() > 0.999, (inr.mean(), decided[inr].mean())
        if name in ("exact", "up", "down"):
            # within an ulp or two of tau only the literal test may decide
            assert decided.mean() < 0.01, (name, decided.mean())


def test_screen_zero_velocity_and_out_of_range(shim):
    # |u| = 0: no fly-by bound; the free-fall term alone decides
    s = Particles(x=np.array([0.0, 1e-3]), y=np.zeros(2), z=np.zeros(2), vx=np.zeros(2), vy=np.zeros(2),
                  vz=np.zeros(2), m=np.array([1e-3, 1e-3]))
    p = oracle.Params(eta=0.01)
    tau = oracle.pair_timesteps(s, np.array([0]), np.array([1]), p)[0]
    for h, want in ((tau * 2, EDGE), (tau / 2, NO)):
        assert _decide(shim, s, [0], [1], [h], 0.01, 0.0, 1.0)[0] == want
    # coincident particles and thresholds outside the certified range go to the literal test
    s0 = Particles(x=np.zeros(2), y=np.zeros(2), z=np.zeros(2), vx=np.array([0.0, 1.0]), vy=np.zeros(2),
                   vz=np.zeros(2), m=np.ones(2))
    assert _decide(shim, s0, [0], [1], [0.1], 0.01, 0.0, 1.0)[0] == UNSURE
    assert _decide(shim, s, [0], [1], [2.0 ** -120], 0.01, 0.0, 1.0)[0] == UNSURE


def _far_cases(rng, tau, n):
    """Thresholds where a far-pair test is most exposed: just above tau (the
    test must not certify "no edge" for a pair whose tau is below h), at tau
    itself, and spread over decades on both sides."""
    return {
        "just_above": tau * (1.0 + rng.integers(1, 400, n) * 2.0 ** -52),
        "up": np.nextafter(tau, np.inf),
        "exact": tau.copy(),
        "x1.001": tau * 1.001,
        "x0.5": tau * 0.5,
        "random": tau * 10.0 ** rng.uniform(-3, 3, n),
    }


@pytest.mark.parametrize("form", FAR_FORMS)
@pytest.mark.parametrize("eta,eps2,G", [(0.01, 0.0, 1.0), (0.3, 0.0, 1.0), (1.0, 1e-8, 4.3e-3),
                                         (0.003, 0.0, 1.0)])
def test_far_test_never_contradicts_literal_test(shim, eta, eps2, G, form):
    """Whenever the far-pair test certifies "no edge", the oracle's literal
    tau is >= h; far from the threshold it certifies most pairs."""
    rng = np.random.default_rng(9105 + int(eta * 1000))
    n = 40000
    s, pi, pj = _pairs_state(rng, n)
    p = oracle.Params(eta=eta, eps2=eps2, G=G)
    tau = oracle.pair_timesteps(s, pi, pj, p)
    ok = (tau > 0) & np.isfinite(tau)
    for name, h in _far_cases(rng, tau, n).items():
        sel = ok & (h > 0) & np.isfinite(h)
        far = _far(shim, s, pi[sel], pj[sel], h[sel], eta, eps2, G, form)
        bad = far & (tau[sel] < h[sel])
        assert not bad.any(), f"{name}: {bad.sum()} pairs certified far with tau < h"
    # h well below every pair's tau: the test certifies the bulk of the pairs
    h = tau / 64.0
    sel = ok & (h >= 2.0 ** -60)
    far = _far(shim, s, pi[sel], pj[sel], h[sel], eta, eps2, G, form)
    assert far.mean() > 0.5, far.mean()


@pytest.mark.parametrize("form", FAR_FORMS)
def test_far_test_with_cut_margin_is_caught(shim_cut, form):
    """Planted mistake: the far-pair header built with its margin cut to one
    half certifies pairs whose tau lies just below h; the same cases find it.
    (The conditions are sufficient ones, tight only at corners of the input
    space, so cuts of a few per cent leave these random pairs decided alike.)"""
    rng = np.random.default_rng(11)
    n = 40000
    s, pi, pj = _pairs_state(rng, n)
    p = oracle.Params(eta=0.01)
    tau = oracle.pair_timesteps(s, pi, pj, p)
    ok = (tau > 0) & np.isfinite(tau)
    wrong = 0
    for name, h in _far_cases(rng, tau, n).items():
        sel = ok & (h > 0) & np.isfinite(h)
        far = _far(shim_cut, s, pi[sel], pj[sel], h[sel], 0.01, 0.0, 1.0, form)
        wrong += int((far & (tau[sel] < h[sel])).sum())
    assert wrong > 0


@pytest.mark.parametrize("form", FAR_FORMS)
def test_far_test_sweep_like_pairs(shim, form):
    """Pairs of a Plummer sphere at the pivot steps of the deep levels: the
    test agrees with the literal decision wherever it decides, and decides
    most pairs at small h."""
    from synth import plummer
    s = plummer(3000, 5, masses="salpeter")
    p = oracle.Params(eta=0.01)
    rng = np.random.default_rng(3)
    pi = rng.integers(0, s.n, 60000).astype(np.int32)
    pj = ((pi + 1 + rng.integers(0, s.n - 1, 60000)) % s.n).astype(np.int32)
    tau = oracle.pair_timesteps(s, pi, pj, p)
    for k in range(0, 12, 2):
        h = np.full(len(pi), 2.0 ** -(6 + k))
        far = _far(shim, s, pi, pj, h, 0.01, 0.0, 1.0, form)
        assert not (far & (tau < h)).any(), k
        if k >= 6:
            assert far.mean() > 0.9, (k, far.mean())
