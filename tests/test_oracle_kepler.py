"""Pins of the oracle's two-body flow (eq. 10) and of CC_KEPLER (Sec. 2.2,
last paragraph; Sec. 3.2; Table 1).

The universal-variable solution is checked against the classical one,
written out independently: Kepler's equation in the eccentric (elliptic) or
hyperbolic anomaly, solved with mpmath at 40 digits, and the orbit's position
and velocity as closed forms of that anomaly.  Then invariants, time
reversal and composition of the flow, and the integrator with the option on:
an isolated binary is advanced exactly, sets without two-body components are
untouched by the option, momenta are conserved."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
import synth
from synth import Particles

mp.mp.dps = 40


def classical_state(mu, a, e, M):
    """Position and velocity in the orbital plane (pericentre on +x, motion
    counter-clockwise) at mean anomaly M, from the eccentric anomaly E
    (E - e sin E = M, e < 1) or the hyperbolic anomaly F (e sinh F - F = M,
    e > 1); a > 0 is the semi-major axis (its magnitude for e > 1)."""
    mu, a, e, M = mp.mpf(mu), mp.mpf(a), mp.mpf(e), mp.mpf(M)
    k = mp.sqrt(mu / a)
    if e < 1:
        E = mp.findroot(lambda E: E - e * mp.sin(E) - M, M + e * mp.sin(M))
        d = 1 - e * mp.cos(E)
        r = [a * (mp.cos(E) - e), a * mp.sqrt(1 - e * e) * mp.sin(E), 0]
        v = [-k * mp.sin(E) / d, k * mp.sqrt(1 - e * e) * mp.cos(E) / d, 0]
    else:
        F = mp.findroot(lambda F: e * mp.sinh(F) - F - M, mp.asinh(M / e))
        d = e * mp.cosh(F) - 1
        r = [a * (e - mp.cosh(F)), a * mp.sqrt(e * e - 1) * mp.sinh(F), 0]
        v = [-k * mp.sinh(F) / d, k * mp.sqrt(e * e - 1) * mp.cosh(F) / d, 0]
    return np.array([float(x) for x in r]), np.array([float(x) for x in v])


def mean_motion(mu, a):
    return math.sqrt(mu / a ** 3)


@pytest.mark.parametrize("e", [0.0, 0.5, 0.9, 0.999])
@pytest.mark.parametrize("M0,periods", [(0.3, 0.37), (2.5, 1.0), (0.0, 12.25), (5.9, 101.6)])
def test_kepler_elliptic_against_anomaly_solution(e, M0, periods):
    mu, a = 0.7, 0.013
    n = mean_motion(mu, a)
    dt = periods * 2 * math.pi / n
    r0, v0 = classical_state(mu, a, e, M0)
    r, v = oracle.kepler(mu, r0, v0, dt)
    rw, vw = classical_state(mu, a, e, M0 + n * dt)
    # the phase after many periods carries the rounding of dt, n and the
    # period reduction: a few ulps of the phase per period
    tol = 1e-13 * (1 + periods)
    scale_r = a * (1 + e)
    scale_v = math.sqrt(mu / a) * math.sqrt((1 + e) / max(1 - e, 1e-300))
    assert np.max(np.abs(r - rw)) <= tol * scale_r / max(1 - e, 1e-3)
    assert np.max(np.abs(v - vw)) <= tol * scale_v / max(1 - e, 1e-3)


@pytest.mark.parametrize("e", [1.2, 3.0])
@pytest.mark.parametrize("M0,dM", [(0.0, 0.5), (-4.0, 6.0), (1.0, 40.0)])
def test_kepler_hyperbolic_against_anomaly_solution(e, M0, dM):
    mu, a = 1.3, 0.05
    n = mean_motion(mu, a)
    r0, v0 = classical_state(mu, a, e, M0)
    r, v = oracle.kepler(mu, r0, v0, dM / n)
    rw, vw = classical_state(mu, a, e, M0 + dM)
    assert np.max(np.abs(r - rw)) <= 1e-12 * np.linalg.norm(rw)
    assert np.max(np.abs(v - vw)) <= 1e-12 * max(np.linalg.norm(vw), math.sqrt(mu / a))


def test_kepler_circular_is_a_rotation():
    """A circular orbit of radius R: after time t the radius vector is turned
    by n t, the velocity with it."""
    mu, R = 2.0, 0.5
    n = math.sqrt(mu / R ** 3)
    for t in (0.1, 1.0, 17.3, -2.2):
        r, v = oracle.kepler(mu, [R, 0, 0], [0, R * n, 0], t)
        assert np.allclose(r, [R * math.cos(n * t), R * math.sin(n * t), 0], rtol=0, atol=1e-13 * R * (1 + abs(n * t)))
        assert np.allclose(v, [-R * n * math.sin(n * t), R * n * math.cos(n * t), 0], rtol=0,
                           atol=1e-13 * R * n * (1 + abs(n * t)))


def _energy_L(mu, r, v):
    return 0.5 * v @ v - mu / np.linalg.norm(r), np.cross(r, v)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_kepler_invariants_reversal_and_composition(seed):
    rng = np.random.default_rng(seed)
    for _ in range(40):
        mu = 10.0 ** rng.uniform(-6, 1)
        r0 = rng.normal(size=3) * 10.0 ** rng.uniform(-5, 0)
        vesc = math.sqrt(2 * mu / np.linalg.norm(r0))
        v0 = rng.normal(size=3) / math.sqrt(3) * vesc * rng.uniform(0.05, 1.6)
        E0, L0 = _energy_L(mu, r0, v0)
        tscale = np.linalg.norm(r0) / np.linalg.norm(v0)
        t = tscale * 10.0 ** rng.uniform(-2, 2)
        r1, v1 = oracle.kepler(mu, r0, v0, t)
        E1, L1 = _energy_L(mu, r1, v1)
        assert abs(E1 - E0) <= 1e-10 * (abs(E0) + 0.5 * v0 @ v0)
        assert np.linalg.norm(L1 - L0) <= 1e-10 * np.linalg.norm(L0)
        # time reversal: back by -t
        rb, vb = oracle.kepler(mu, r1, v1, -t)
        assert np.linalg.norm(rb - r0) <= 1e-9 * np.linalg.norm(r0)
        # composition: t1 then t2 equals t1 + t2
        ra, va = oracle.kepler(mu, *oracle.kepler(mu, r0, v0, 0.3 * t), 0.7 * t)
        assert np.linalg.norm(ra - r1) <= 1e-9 * max(np.linalg.norm(r1), np.linalg.norm(r0))


def test_kepler_errors():
    with pytest.raises(oracle.OracleError):
        oracle.kepler(0.0, [1, 0, 0], [0, 1, 0], 1.0)
    with pytest.raises(oracle.OracleError):
        oracle.kepler(1.0, [0, 0, 0], [0, 1, 0], 1.0)


def binary(m1, m2, a, e, M0, X0=(0.1, -0.2, 0.3), V0=(0.01, 0.02, -0.03)):
    r, v = classical_state(m1 + m2, a, e, M0)
    M = m1 + m2
    pos = np.array([-m2 / M * r, m1 / M * r]) + np.array(X0)
    vel = np.array([-m2 / M * v, m1 / M * v]) + np.array(V0)
    return Particles.from_arrays(pos, vel, np.array([m1, m2]))


def test_cc_kepler_isolated_binary_is_exact():
    """A bound pair whose pair step is below dt0 forms one component: with
    the option on it is advanced by two Kepler solutions of dt0/2 per global
    step, so after 64 steps it sits where the closed form puts it (plain CC
    recurses and carries the integrator's second-order error instead)."""
    m1, m2, a, e, M0 = 0.3, 0.7, 0.01, 0.6, 1.1
    s = binary(m1, m2, a, e, M0)
    p = oracle.Params(eta=0.01, kepler=1)
    dt = 1 / 64
    ref = s.copy()
    rc, st = oracle.evolve(ref, dt, 1.0, p)
    assert st["kepler_solves"] == 2 * 64 and st["splits"] == 64 and st["kick_pairs"] == 0
    n = mean_motion(1.0, a)
    rw, vw = classical_state(1.0, a, e, M0 + n * 1.0)
    rel = np.array([ref.x[1] - ref.x[0], ref.y[1] - ref.y[0], ref.z[1] - ref.z[0]])
    assert np.linalg.norm(rel - rw) <= 1e-10 * a
    # the centre of mass moved uniformly
    com = (m1 * ref.pos()[0] + m2 * ref.pos()[1]) / (m1 + m2)
    assert np.allclose(com, np.array([0.1, -0.2, 0.3]) + np.array([0.01, 0.02, -0.03]) * 1.0, rtol=0, atol=1e-14)
    plain = s.copy()
    oracle.evolve(plain, dt, 1.0, oracle.Params(eta=0.01))
    relp = np.array([plain.x[1] - plain.x[0], plain.y[1] - plain.y[0], plain.z[1] - plain.z[0]])
    assert np.linalg.norm(relp - rw) > 100 * np.linalg.norm(rel - rw)


def test_cc_kepler_same_as_cc_without_two_body_components():
    """All bodies slow at dt0 (no component at all): the option changes nothing, bit for bit."""
    rng = np.random.default_rng(4)
    n = 60
    s = Particles.from_arrays(rng.uniform(-1, 1, (n, 3)) * 10, rng.normal(size=(n, 3)) * 1e-3,
                              rng.uniform(1, 2, n) * 1e-12)
    a, b = s.copy(), s.copy()
    _, sa = oracle.evolve(a, 1 / 64, 4 / 64, oracle.Params(eta=0.01))
    _, sb = oracle.evolve(b, 1 / 64, 4 / 64, oracle.Params(eta=0.01, kepler=1))
    assert sb["kepler_solves"] == 0
    for u, v in zip(a.arrays(), b.arrays()):
        np.testing.assert_array_equal(u, v)


def test_cc_kepler_conserves_momenta_with_binaries():
    s = synth.workload(5, n=600)
    p = oracle.Params(eta=0.01, kepler=1)
    d0 = oracle.diagnostics(s)
    ref = s.copy()
    _, st = oracle.evolve(ref, 1 / 64, 2 / 64, p)
    assert st["kepler_solves"] > 0
    d1 = oracle.diagnostics(ref)
    pscale = np.sum(s.m * np.linalg.norm(s.vel(), axis=1))
    assert np.linalg.norm(d1["P"] - d0["P"]) <= 1e-14 * pscale
    lscale = np.sum(s.m * np.linalg.norm(np.cross(s.pos(), s.vel()), axis=1))
    assert np.linalg.norm(d1["L"] - d0["L"]) <= 1e-13 * lscale
    assert abs(d1["energy"] / d0["energy"] - 1) < 1e-6


def test_cc_kepler_rejects_softening():
    s = synth.plummer(20, 1)
    with pytest.raises(oracle.OracleError) as e:
        oracle.evolve(s, 1 / 64, 1 / 64, oracle.Params(eps2=1e-6, kepler=1))
    assert e.value.code == oracle.CCO_ERR_ARG
