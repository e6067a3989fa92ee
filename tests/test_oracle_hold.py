"""Pins of the oracle's HOLD split (Sec. 2.1, eqs. 11-17): the particle time
step tau(i) = min_j tau(i,j), the fast set F recursed into as one set, the
kick of every pair with a slow member; its relation to the CC split (the
paper's example of isolated fast subsystems, Sec. 2.1), exact work counts,
second order and conservation."""
import math

import numpy as np
import pytest

import oracle
from synth import Particles, plummer


def circular_binaries(K, a, spacing, mass=1.0, seed=3):
    """K equal circular binaries of semi-major axis a (separation a), centres
    on a line `spacing` apart and at rest: every binary's pair step is
    eta a^(3/2) / sqrt(G mass), every pair across binaries is slow."""
    rng = np.random.default_rng(seed)
    pos, vel = [], []
    v = math.sqrt(mass / a) / 2.0      # each member's speed about the common centre
    for k in range(K):
        c = np.array([k * spacing, 0.0, 0.0])
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        w = np.cross(d, rng.normal(size=3))
        w /= np.linalg.norm(w)
        pos += [c - 0.5 * a * d, c + 0.5 * a * d]
        vel += [-v * w, v * w]
    return Particles.from_arrays(np.array(pos), np.array(vel), np.full(2 * K, mass / 2.0))


def test_hold_equals_cc_with_one_fast_subsystem():
    """One tight binary in a slow field: at every level F is the one
    non-trivial component, so HOLD and CC make the same drifts and kicks in
    the same order, bit for bit."""
    rng = np.random.default_rng(8)
    n = 40
    pos = rng.uniform(-1, 1, (n, 3)) * 20
    vel = rng.normal(size=(n, 3)) * 1e-3
    m = rng.uniform(1, 2, n) * 1e-10
    pos[7] = pos[3] + np.array([1e-3, 0, 0])
    vel[3] = [0, 0.5, 0]
    vel[7] = [0, -0.5, 0]
    m[3] = m[7] = 0.25
    s = Particles.from_arrays(pos, vel, m)
    a, b = s.copy(), s.copy()
    _, sa = oracle.evolve(a, 1 / 64, 2 / 64, oracle.Params(eta=0.01))
    _, sb = oracle.evolve(b, 1 / 64, 2 / 64, oracle.Params(eta=0.01, hold=1))
    for u, v in zip(a.arrays(), b.arrays()):
        np.testing.assert_array_equal(u, v)
    for k in ("kick_pairs", "drifts", "components", "splits", "max_depth_seen"):
        assert sa[k] == sb[k], k
    assert sb["tau_evals"] >= sa["tau_evals"]   # HOLD evaluates every pair; the BFS at most as many


@pytest.mark.parametrize("K", [3, 5])
def test_hold_isolated_binaries_become_a_shared_step(K):
    """K isolated identical circular binaries whose pair step lies between
    dt0/2^L and dt0/2^(L-1): CC kicks the pairs across binaries once per
    global step (at the top) and each binary's own pair 2^L times (its
    leaves); HOLD keeps every particle in F down to depth L, so every pair is
    kicked 2^L times and every split evaluates all pairs (Sec. 2.1)."""
    mass, dt = 1.0, 1 / 64
    L = 4
    # eta a^1.5 / sqrt(mass) = 0.75 dt0 / 2^(L-1): inside (dt0/2^L, dt0/2^(L-1))
    eta = 0.01
    a = (0.75 * dt / 2 ** (L - 1) * math.sqrt(mass) / eta) ** (2 / 3)
    s = circular_binaries(K, a, spacing=50.0, mass=mass)
    n = 2 * K
    P2 = n * (n - 1) // 2
    cc, ho = s.copy(), s.copy()
    _, scc = oracle.evolve(cc, dt, dt, oracle.Params(eta=eta))
    _, sho = oracle.evolve(ho, dt, dt, oracle.Params(eta=eta, hold=1))
    assert scc["max_depth_seen"] == L and sho["max_depth_seen"] == L
    assert sho["kick_pairs"] == 2 ** L * P2
    assert scc["kick_pairs"] == (P2 - K) + K * 2 ** L
    assert sho["tau_evals"] == (2 ** (L + 1) - 1) * P2
    assert sho["drifts"] == 2 * n * 2 ** L and scc["drifts"] == sho["drifts"]


def test_hold_all_slow_is_leapfrog_like_cc():
    rng = np.random.default_rng(11)
    n = 30
    s = Particles.from_arrays(rng.uniform(-1, 1, (n, 3)) * 10, rng.normal(size=(n, 3)) * 1e-3,
                              rng.uniform(1, 2, n) * 1e-12)
    a, b = s.copy(), s.copy()
    oracle.evolve(a, 1 / 64, 3 / 64, oracle.Params(eta=0.01))
    _, st = oracle.evolve(b, 1 / 64, 3 / 64, oracle.Params(eta=0.01, hold=1))
    assert st["components"] == 0 and st["tau_evals"] == 3 * n * (n - 1) // 2
    for u, v in zip(a.arrays(), b.arrays()):
        np.testing.assert_array_equal(u, v)


def test_hold_second_order_in_eta():
    """Energy error of a softened 64-body Plummer sphere to t = 1 falls as
    eta^2 (Sec. 3.1: both splits are second-order schemes)."""
    s0 = plummer(64, 5)
    errs = []
    etas = (0.04, 0.02, 0.01)
    for eta in etas:
        s = s0.copy()
        p = oracle.Params(eta=eta, eps2=(1 / 64) ** 2, hold=1)
        e0 = oracle.diagnostics(s, p)["energy"]
        oracle.evolve(s, 1 / 16, 1.0, p)
        errs.append(abs(oracle.diagnostics(s, p)["energy"] / e0 - 1))
    slopes = [math.log(errs[i] / errs[i + 1]) / math.log(etas[i] / etas[i + 1]) for i in range(2)]
    assert all(1.4 < k < 2.8 for k in slopes), (errs, slopes)


def test_hold_conserves_momenta():
    s = plummer(128, 9, masses="salpeter")
    p = oracle.Params(eta=0.01, hold=1)
    d0 = oracle.diagnostics(s)
    r = s.copy()
    _, st = oracle.evolve(r, 1 / 64, 4 / 64, p)
    assert st["components"] > 0
    d1 = oracle.diagnostics(r)
    pscale = np.sum(s.m * np.linalg.norm(s.vel(), axis=1))
    assert np.linalg.norm(d1["P"] - d0["P"]) <= 1e-15 * pscale
    lscale = np.sum(s.m * np.linalg.norm(np.cross(s.pos(), s.vel()), axis=1))
    assert np.linalg.norm(d1["L"] - d0["L"]) <= 1e-14 * lscale


def test_hold_with_kepler_is_rejected():
    s = plummer(10, 1)
    with pytest.raises(oracle.OracleError) as e:
        oracle.evolve(s, 1 / 64, 1 / 64, oracle.Params(hold=1, kepler=1))
    assert e.value.code == oracle.CCO_ERR_ARG
