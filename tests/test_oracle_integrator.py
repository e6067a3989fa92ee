"""Pins of the oracle's kick/drift operators (eqs. 6, 8, 9) and of the
recursive CC integrator (eqs. 26-31, Fig. 2): closed forms, exact special
cases, conservation laws (Sec. 1, Sec. 3.1), second order (Sec. 3.1),
approximate reversibility and the error paths."""
import math

import numpy as np
import pytest

import oracle
from synth import Particles, plummer


def line_set(xs, ms):
    n = len(xs)
    pos = np.zeros((n, 3))
    pos[:, 0] = xs
    return Particles.from_arrays(pos, np.zeros((n, 3)), np.array(ms, float))


# ---------------------------------------------------------------- kick/drift

def test_kick_two_body_closed_form():
    s = line_set([0.0, 2.0], [0.25, 0.75])
    oracle.kick(s, 0.5)
    # dv_0 = h G m_1 / r^2 toward 1, dv_1 = -h G m_0 / r^2
    assert s.vx[0] == pytest.approx(0.5 * 0.75 / 4.0, rel=1e-15)
    assert s.vx[1] == pytest.approx(-0.5 * 0.25 / 4.0, rel=1e-15)
    assert s.vy[0] == 0.0 and s.vz[1] == 0.0


def test_kick_softened_closed_form():
    s = line_set([0.0, 1.0], [0.5, 0.5])
    oracle.kick(s, 1.0, p=oracle.Params(eps2=3.0))
    # (r^2 + eps^2)^(3/2) = 8
    assert s.vx[0] == pytest.approx(0.5 / 8.0, rel=1e-15)


def test_kick_respects_labels():
    # collinear 0,1,3,6 with labels {0,1},{2,3}: particle 0 feels only 2 and 3
    ms = [0.1, 0.2, 0.3, 0.4]
    s = line_set([0.0, 1.0, 3.0, 6.0], ms)
    pairs = oracle.kick(s, 1.0, label=np.array([0, 0, 2, 2]))
    assert pairs == 4
    assert s.vx[0] == pytest.approx(0.3 / 9.0 + 0.4 / 36.0, rel=1e-15)
    assert s.vx[3] == pytest.approx(-(0.1 / 36.0 + 0.2 / 25.0), rel=1e-15)


def test_octahedron_centre_feels_nothing():
    pts = [[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]]
    s = Particles.from_arrays(np.array(pts, float), np.zeros((7, 3)), np.full(7, 1 / 7))
    a = oracle.accel(s, np.array([0]))
    assert np.all(a == 0.0)


def test_kick_conserves_momentum():
    rng = np.random.default_rng(2)
    n = 80
    s = Particles.from_arrays(rng.normal(size=(n, 3)), rng.normal(size=(n, 3)), rng.uniform(0.1, 1, n))
    v0 = s.vel().copy()
    lab = rng.integers(0, 5, n)
    oracle.kick(s, 0.01, label=lab)
    dp = (s.m[:, None] * (s.vel() - v0)).sum(0)
    scale = np.sum(s.m[:, None] * np.abs(s.vel() - v0))
    assert np.all(np.abs(dp) <= 1e-15 * scale)


def test_kick_equals_accel_bitwise():
    rng = np.random.default_rng(4)
    n = 33
    s = Particles.from_arrays(rng.normal(size=(n, 3)), np.zeros((n, 3)), rng.uniform(0.1, 1, n))
    a = oracle.accel(s)
    oracle.kick(s, 1.0)
    np.testing.assert_array_equal(s.vel(), a)
    ac = oracle.accel(s, compensated=True)
    np.testing.assert_allclose(a, ac, rtol=1e-13, atol=1e-13 * np.abs(ac).max())


def test_drift_exact():
    s = line_set([1.0, 2.0, 3.0], [1, 1, 1])
    s.vx[:] = [0.5, -0.25, 1.0]
    oracle.drift(s, 2.0, mask=np.array([1, 0, 1], np.uint8))
    np.testing.assert_array_equal(s.x, [2.0, 2.0, 5.0])


def test_kick_zero_separation_is_error():
    s = line_set([1.0, 1.0], [0.5, 0.5])
    with pytest.raises(oracle.OracleError) as e:
        oracle.kick(s, 1.0)
    assert e.value.code == oracle.CCO_ERR_NONFINITE
    assert np.all(s.vx == 0.0)


# ---------------------------------------------------------------- integrator

def test_single_component_halving_identity():
    """If all particles form one component at dt0, evolve(dt0) is exactly two
    calls at dt0/2 (R is empty, eqs. 26-27)."""
    s = plummer(24, 31)
    p = oracle.Params(eta=0.05)
    dt0 = 1.0
    lab, nt, _ = oracle.split_labels(s, dt0, p)
    assert nt == 1 and np.all(lab == 0)
    a, b = s.copy(), s.copy()
    oracle.evolve(a, dt0, dt0, p)
    oracle.evolve(b, dt0 / 2, dt0, p)
    for u, v in zip(a.arrays(), b.arrays()):
        np.testing.assert_array_equal(u, v)


def _leapfrog(s, h, G=1.0, eps2=0.0):
    """Plain DKD leapfrog in Python floats (drift h/2, all pair kicks, drift h/2)."""
    n = len(s.m)
    hh = 0.5 * h
    for i in range(n):
        s.x[i] += hh * s.vx[i]; s.y[i] += hh * s.vy[i]; s.z[i] += hh * s.vz[i]
    ax = [0.0] * n; ay = [0.0] * n; az = [0.0] * n
    for i in range(n):
        for j in range(i + 1, n):
            dx = s.x[j] - s.x[i]; dy = s.y[j] - s.y[i]; dz = s.z[j] - s.z[i]
            r2 = ((dx * dx + dy * dy) + dz * dz) + eps2
            f = G / (r2 * math.sqrt(r2))
            mj, mi = s.m[j] * f, s.m[i] * f
            ax[i] += mj * dx; ay[i] += mj * dy; az[i] += mj * dz
            ax[j] -= mi * dx; ay[j] -= mi * dy; az[j] -= mi * dz
    for i in range(n):
        s.vx[i] += h * ax[i]; s.vy[i] += h * ay[i]; s.vz[i] += h * az[i]
    for i in range(n):
        s.x[i] += hh * s.vx[i]; s.y[i] += hh * s.vy[i]; s.z[i] += hh * s.vz[i]


def test_all_slow_is_global_leapfrog():
    """With every tau >= dt0 all particles are in R and one CC step is the
    textbook DKD leapfrog (eq. 30 with H_C empty)."""
    rng = np.random.default_rng(6)
    n = 7
    s = Particles.from_arrays(rng.uniform(-1, 1, (n, 3)) * 10, rng.normal(size=(n, 3)) * 1e-3,
                              rng.uniform(1, 2, n) * 1e-12)
    p = oracle.Params(eta=0.01)
    dt0 = 1.0 / 64
    lab, nt, _ = oracle.split_labels(s, dt0, p)
    assert nt == 0
    a, b = s.copy(), s.copy()
    rc, st = oracle.evolve(a, dt0, 4 * dt0, p)
    for _ in range(4):
        _leapfrog(b, dt0)
    for u, v in zip(a.arrays(), b.arrays()):
        np.testing.assert_array_equal(u, v)
    assert st["max_depth_seen"] == 0 and st["kick_pairs"] == 4 * n * (n - 1) // 2
    assert st["drifts"] == 4 * 2 * n


def kepler_binary(e, a=1.0, m1=0.5, m2=0.5):
    """Relative orbit started at pericentre in the x-y plane, COM at rest."""
    mu = m1 + m2
    rp = a * (1 - e)
    vp = math.sqrt(mu / a * (1 + e) / (1 - e))
    q = np.array([rp, 0.0, 0.0])
    u = np.array([0.0, vp, 0.0])
    pos = np.stack([q * m2 / mu, -q * m1 / mu])
    vel = np.stack([u * m2 / mu, -u * m1 / mu])
    return Particles.from_arrays(pos, vel, np.array([m1, m2]))


def _energy(s):
    d = oracle.diagnostics(s)
    return d["energy"]


@pytest.mark.parametrize("e", [0.0, 0.5, 0.9])
def test_kepler_orbit_second_order(e):
    """After one period the exact orbit is back at pericentre; the CC
    integrator's position error shrinks as eta^2 and its energy error stays
    bounded (Sec. 3.1)."""
    P = 2 * math.pi
    dt0 = P / 16
    errs = []
    for eta in (0.02, 0.01, 0.005):
        s0 = kepler_binary(e)
        s = s0.copy()
        rc, st = oracle.evolve(s, dt0, P, oracle.Params(eta=eta))
        q = s.pos()[0] - s.pos()[1]
        q0 = s0.pos()[0] - s0.pos()[1]
        errs.append(np.linalg.norm(q - q0) / np.linalg.norm(q0))
        assert abs(_energy(s) / _energy(s0) - 1) < 50 * eta ** 2
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 2.5 < r1 < 6.5 and 2.5 < r2 < 6.5, errs


def test_kepler_energy_error_bounded_over_many_orbits():
    """The time-symmetrised criterion keeps the energy error of an eccentric
    orbit small over many orbits (no secular drift at the level a one-sided
    step choice produces, ~4e-5 per orbit here), shrinking with eta."""
    P = 2 * math.pi
    worst = []
    for eta in (0.01, 0.005):
        s0 = kepler_binary(0.5)
        s = s0.copy()
        p = oracle.Params(eta=eta)
        w = 0.0
        for k in range(8):
            oracle.evolve(s, P / 16, P, p)
            w = max(w, abs(_energy(s) / _energy(s0) - 1))
        worst.append(w)
    assert worst[0] < 1e-6 and worst[1] < worst[0] / 3, worst


def test_momentum_and_angular_momentum_conserved():
    """Kicks come in equal and opposite pairs, so P and L only change by
    rounding (Sec. 1, Sec. 3.1)."""
    s0 = plummer(64, 3)
    s = s0.copy()
    p = oracle.Params(eta=0.01)
    rc, st = oracle.evolve(s, 1 / 64, 1 / 8, p)
    d0, d1 = oracle.diagnostics(s0), oracle.diagnostics(s)
    pscale = np.sum(s.m * np.linalg.norm(s.vel(), axis=1))
    lscale = np.sum(s.m * np.linalg.norm(s.pos(), axis=1) * np.linalg.norm(s.vel(), axis=1))
    assert np.all(np.abs(d1["P"] - d0["P"]) < 1e-14 * pscale)
    assert np.all(np.abs(d1["L"] - d0["L"]) < 1e-14 * lscale)
    # centre of mass moves with the (tiny) total momentum
    assert np.all(np.abs(d1["com"] - d0["com"] - d0["P"] / d0["mass"] / 8) < 1e-14)
    assert st["kick_pairs"] > 0 and st["max_depth_seen"] >= 1


def test_energy_error_second_order_in_eta():
    """Energy error vs eta shows second-order behaviour (Sec. 3.1)."""
    s0 = plummer(32, 12)
    p_eps = 1.0 / 64 ** 2
    dt0 = 1 / 16
    errs = []
    for eta in (0.04, 0.02, 0.01):
        s = s0.copy()
        p = oracle.Params(eta=eta, eps2=p_eps)
        e0 = oracle.diagnostics(s0, p)["energy"]
        worst = 0.0
        for _ in range(8):
            oracle.evolve(s, dt0, dt0, p)
            worst = max(worst, abs(oracle.diagnostics(s, p)["energy"] / e0 - 1))
        errs.append(worst)
    slopes = [math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])]
    assert 1.3 < np.mean(slopes) < 2.7, (errs, slopes)


def test_approximately_time_reversible():
    """Forward, reverse the velocities, forward again: back near the start,
    closer for smaller eta (Sec. 1)."""
    s0 = plummer(16, 21)
    errs = []
    for eta in (0.02, 0.005):
        p = oracle.Params(eta=eta, eps2=1e-4)
        s = s0.copy()
        oracle.evolve(s, 1 / 16, 1 / 4, p)
        moved = np.linalg.norm(s.pos() - s0.pos())
        for a in (s.vx, s.vy, s.vz):
            a *= -1.0
        oracle.evolve(s, 1 / 16, 1 / 4, p)
        errs.append(np.linalg.norm(s.pos() - s0.pos()) / moved)
    assert errs[0] < 1e-3 and errs[1] < errs[0]


def test_resume_is_bit_identical():
    """No state is carried between global steps: two calls equal one."""
    s0 = plummer(48, 8)
    p = oracle.Params(eta=0.01)
    a, b = s0.copy(), s0.copy()
    oracle.evolve(a, 1 / 64, 1 / 16, p)
    oracle.evolve(b, 1 / 64, 1 / 32, p)
    oracle.evolve(b, 1 / 64, 1 / 32, p)
    for u, v in zip(a.arrays(), b.arrays()):
        np.testing.assert_array_equal(u, v)


def test_two_body_stats():
    s = kepler_binary(0.0)
    p = oracle.Params(eta=0.01)
    rc, st = oracle.evolve(s, 1 / 16, 1 / 16, p)
    # every leaf of the bisection is one pair kick and four half-drifts
    leaves = st["kick_pairs"]
    assert st["drifts"] == 4 * leaves
    # each split of a two-particle set evaluates tau once
    assert st["tau_evals"] == st["splits"]
    assert st["components"] == st["splits"] - leaves


def test_batch_equals_individual_runs():
    parts = [plummer(n, 100 + n) for n in (8, 13, 21)]
    off = np.cumsum([0] + [q.n for q in parts])
    cat = Particles(*(np.concatenate([getattr(q, f) for q in parts])
                      for f in ("x", "y", "z", "vx", "vy", "vz", "m")))
    p = oracle.Params(eta=0.01)
    rc, sts = oracle.evolve_batch(cat, off, 1 / 32, 1 / 8, p)
    for k, q in enumerate(parts):
        r = q.copy()
        rc, st = oracle.evolve(r, 1 / 32, 1 / 8, p)
        assert st == sts[k]
        for u, f in zip(r.arrays(), ("x", "y", "z", "vx", "vy", "vz", "m")):
            np.testing.assert_array_equal(u, getattr(cat, f)[off[k]:off[k + 1]])


def test_error_paths():
    p = oracle.Params(eta=0.01)
    s = plummer(16, 4)
    with pytest.raises(oracle.OracleError) as e:
        oracle.evolve(s.copy(), 1 / 64, 1 / 100, p)        # t_end/dt not an integer
    assert e.value.code == oracle.CCO_ERR_ARG
    with pytest.raises(oracle.OracleError):
        oracle.evolve(s.copy(), 0.0, 1.0, p)
    bad = s.copy()
    bad.m[3] = 0.0
    with pytest.raises(oracle.OracleError) as e:
        oracle.evolve(bad, 1 / 64, 1 / 64, p)
    assert e.value.code == oracle.CCO_ERR_ARG
    bad = s.copy()
    bad.vy[5] = np.nan
    rc, st = oracle.evolve(bad, 1 / 64, 1 / 64, p, raise_on_error=False)
    assert rc == oracle.CCO_ERR_NONFINITE and st["t_reached"] == 0.0
    # depth cap: a tight binary needs many halvings
    b = kepler_binary(0.0, a=1e-3)
    b0 = b.copy()
    rc, st = oracle.evolve(b, 1 / 64, 2 / 64, oracle.Params(eta=0.01, max_depth=3), raise_on_error=False)
    assert rc == oracle.CCO_ERR_DEPTH and st["t_reached"] == 0.0
    for u, v in zip(b.arrays(), b0.arrays()):
        np.testing.assert_array_equal(u, v)
