"""Pins of the oracle's pair time step tau(i,j) (eq. 19) to closed forms,
the exact two-body motion and symmetry -- nothing here re-types the formula.
"""
import math

import numpy as np
import pytest

import oracle
from synth import Particles

from .golden import load_golden


def two_body(q, u, m1=0.5, m2=0.5):
    """Particles 0 and 1 with relative position q = q0 - q1, velocity u = v0 - v1
    (centre of mass at rest at the origin)."""
    q = np.asarray(q, float)
    u = np.asarray(u, float)
    M = m1 + m2
    pos = np.stack([q * (m2 / M), -q * (m1 / M)])
    vel = np.stack([u * (m2 / M), -u * (m1 / M)])
    return Particles.from_arrays(pos, vel, np.array([m1, m2]))


def exact_pair(q, u, m1=0.5, m2=0.5):
    """Two particles with exactly the given coordinate differences (particle 1 at rest at 0)."""
    pos = np.array([q, [0.0, 0.0, 0.0]], float)
    vel = np.array([u, [0.0, 0.0, 0.0]], float)
    return Particles.from_arrays(pos, vel, np.array([m1, m2]))


@pytest.mark.parametrize("a,mu", [(1.0, 1.0), (0.3, 2.0e-3), (1e-4, 1e-5), (7.5, 0.25)])
def test_circular_orbit_closed_form(a, mu):
    # rv = 0, |u| = sqrt(mu/a): both derivatives vanish and t_ff = t_fb = sqrt(a^3/mu)
    p = oracle.Params(eta=0.01)
    s = exact_pair([a, 0.0, 0.0], [0.0, math.sqrt(mu / a), 0.0], mu / 2, mu / 2)
    want = 0.01 * math.sqrt(a ** 3 / mu)
    assert oracle.tau(s, 0, 1, p) == pytest.approx(want, rel=4e-16 * 8)
    parts = oracle.tau_parts(s, 0, 1, p)
    assert parts[1] == 0.0 and parts[3] == 0.0
    assert parts[0] == pytest.approx(math.sqrt(a ** 3 / mu), rel=1e-15)
    assert parts[2] == pytest.approx(math.sqrt(a ** 3 / mu), rel=1e-15)


def test_pair_at_rest_closed_form():
    # zero relative velocity: only the free-fall bound, tau = eta sqrt(r^3/mu)
    p = oracle.Params(eta=0.03)
    s = exact_pair([3.0, 4.0, 0.0], [0.0, 0.0, 0.0], 0.25, 0.75)
    assert oracle.tau(s, 0, 1, p) == pytest.approx(0.03 * math.sqrt(125.0), rel=1e-15)
    assert math.isinf(oracle.tau_parts(s, 0, 1, p)[2])


def test_golden_closed_form_cases():
    for case in load_golden("tau_closed_form.txt"):
        s = exact_pair(case["q"], case["u"], case["m1"], case["m2"])
        p = oracle.Params(eta=case["eta"], eps2=case["eps2"])
        got = oracle.tau(s, 0, 1, p)
        assert got == pytest.approx(case["tau"], rel=2e-15, abs=0.0), case


def test_softening_enters_r():
    # at rest, r^2 = |q|^2 + eps^2: tau = eta sqrt((q^2+eps^2)^(3/2)/mu)
    p = oracle.Params(eta=0.01, eps2=0.75)
    s = exact_pair([0.5, 0.0, 0.0], [0.0, 0.0, 0.0], 0.5, 0.5)
    assert oracle.tau(s, 0, 1, p) == pytest.approx(0.01 * 1.0, rel=1e-15)


def test_bitwise_symmetric():
    rng = np.random.default_rng(3)
    n = 64
    s = Particles.from_arrays(rng.normal(size=(n, 3)), rng.normal(size=(n, 3)), rng.uniform(0.1, 1, n))
    for i, j in rng.integers(0, n, size=(300, 2)):
        if i == j:
            continue
        a, b = oracle.tau(s, int(i), int(j)), oracle.tau(s, int(j), int(i))
        assert a == b or (math.isinf(a) and math.isinf(b))


def test_approaching_shorter_receding_longer():
    # eq. 19: approaching pairs (q.u < 0) get a step shorter than eta*t, receding ones longer
    p = oracle.Params(eta=0.01)
    for sign in (-1.0, 1.0):
        s = exact_pair([1.0, 0.0, 0.0], [sign * 0.3, 0.9, 0.0], 0.5, 0.5)
        parts = oracle.tau_parts(s, 0, 1, p)
        unsym = 0.01 * min(parts[0], parts[2])
        t = oracle.tau(s, 0, 1, p)
        if sign < 0:
            assert t < unsym
        else:
            assert t > unsym


def _kepler_rhs(mu, eps2):
    def f(t, y):
        q, u = y[:3], y[3:]
        r2 = q @ q + eps2
        return np.concatenate([u, -mu * q / r2 ** 1.5])
    return f


@pytest.mark.parametrize("q0,u0,mu,eps2", [
    ([1.0, 0.2, 0.0], [-0.4, 0.9, 0.1], 1.0, 0.0),        # bound, approaching
    ([0.5, -0.3, 0.2], [0.8, 0.5, -0.2], 0.5, 0.0),       # bound, receding
    ([2.0, 1.0, 0.0], [-3.0, 0.5, 0.0], 1.0, 0.0),        # hyperbolic fly-by
    ([0.3, 0.0, 0.1], [0.2, 1.1, 0.0], 0.8, 0.01),        # softened
])
def test_derivatives_match_two_body_motion(q0, u0, mu, eps2):
    """d t_ff/dt and d t_fb/dt (eq. 19) against central differences of
    t_ff = sqrt(r^3/mu), t_fb = r/|u| along the integrated two-body orbit."""
    from scipy.integrate import solve_ivp
    p = oracle.Params(eta=0.01, eps2=eps2, G=1.0)
    s = exact_pair(q0, u0, mu / 2, mu / 2)
    parts = oracle.tau_parts(s, 0, 1, p)
    d = 1e-4
    y0 = np.array(q0 + u0, float)
    sol = solve_ivp(_kepler_rhs(mu, eps2), (0.0, d), y0, method="DOP853", rtol=1e-13, atol=1e-15,
                    dense_output=False, t_eval=[d])
    solm = solve_ivp(_kepler_rhs(mu, eps2), (0.0, -d), y0, method="DOP853", rtol=1e-13, atol=1e-15,
                     t_eval=[-d])

    def tff(y):
        r = math.sqrt(y[:3] @ y[:3] + eps2)
        return math.sqrt(r ** 3 / mu)

    def tfb(y):
        r = math.sqrt(y[:3] @ y[:3] + eps2)
        return r / math.sqrt(y[3:] @ y[3:])

    yp, ym = sol.y[:, -1], solm.y[:, -1]
    assert parts[1] == pytest.approx((tff(yp) - tff(ym)) / (2 * d), rel=1e-6, abs=1e-9)
    assert parts[3] == pytest.approx((tfb(yp) - tfb(ym)) / (2 * d), rel=1e-6, abs=1e-9)
    assert parts[0] == pytest.approx(tff(y0), rel=1e-14)
    assert parts[2] == pytest.approx(tfb(y0), rel=1e-14)


def test_nonpositive_denominator_drops_that_term():
    # eta = 1, radial recession at the circular speed: the fly-by denominator
    # is 0, so the free-fall term alone sets the step; faster recession drops
    # the free-fall term instead
    p = oracle.Params(eta=1.0)
    s = exact_pair([1.0, 0.0, 0.0], [1.0, 0.0, 0.0], 0.5, 0.5)
    parts = oracle.tau_parts(s, 0, 1, p)
    assert 1 - 0.5 * parts[3] <= 0 < 1 - 0.5 * parts[1]
    assert oracle.tau(s, 0, 1, p) == pytest.approx(4.0, rel=1e-15)
    s = exact_pair([1.0, 0.0, 0.0], [5.0, 0.0, 0.0], 0.5, 0.5)
    parts = oracle.tau_parts(s, 0, 1, p)
    assert 1 - 0.5 * parts[1] <= 0 < 1 - 0.5 * parts[3]
    assert oracle.tau(s, 0, 1, p) == pytest.approx(5.0 / 12.0, rel=1e-15)


def test_eta_scales_the_symmetrised_step():
    # the symmetrisation acts on eta*t: for small eta the correction is small,
    # tau / (eta t) -> 1, and the step grows less than linearly in eta for a
    # receding pair (denominator 1 - eta t'/2 shrinks as eta grows)
    s = exact_pair([1.0, 0.0, 0.0], [0.3, 1.2, 0.0], 0.5, 0.5)
    parts = oracle.tau_parts(s, 0, 1, oracle.Params(eta=1.0))
    base = min(parts[0], parts[2])
    r_small = oracle.tau(s, 0, 1, oracle.Params(eta=1e-6)) / (1e-6 * base)
    assert r_small == pytest.approx(1.0, abs=1e-5)
    t1 = oracle.tau(s, 0, 1, oracle.Params(eta=0.01))
    t2 = oracle.tau(s, 0, 1, oracle.Params(eta=0.02))
    assert t2 > 2 * t1


def test_tau_always_finite_for_separated_pairs():
    # with w = |u| / sqrt(mu/r) and c = cos(q,u): eta t_ff' = 1.5 eta w c and
    # eta t_fb' = eta c (1 + 1/w^2) cannot both reach 2 for eta <= 1, so one
    # term always bounds tau
    rng = np.random.default_rng(11)
    n = 200
    s = Particles.from_arrays(rng.normal(size=(n, 3)) * rng.uniform(1e-3, 10, (n, 1)),
                              rng.normal(size=(n, 3)) * rng.uniform(1e-3, 100, (n, 1)),
                              rng.uniform(1e-6, 1, n))
    pi, pj = np.triu_indices(n, 1)
    t = oracle.pair_timesteps(s, pi.astype(np.int32), pj.astype(np.int32))
    assert np.all(np.isfinite(t)) and np.all(t > 0)


def test_coincident_pair_zero_step():
    p = oracle.Params(eta=0.01, eps2=0.0)
    s = exact_pair([0.0, 0.0, 0.0], [1.0, 0.0, 0.0], 0.5, 0.5)
    assert oracle.tau(s, 0, 1, p) == 0.0


def test_pair_timesteps_list_matches_single_calls():
    rng = np.random.default_rng(5)
    n = 50
    s = Particles.from_arrays(rng.normal(size=(n, 3)), rng.normal(size=(n, 3)), rng.uniform(0.1, 1, n))
    pi = rng.integers(0, n, 200).astype(np.int32)
    pj = rng.integers(0, n, 200).astype(np.int32)
    t = oracle.pair_timesteps(s, pi, pj)
    for k in range(200):
        if pi[k] == pj[k]:
            assert t[k] == 0.0
        else:
            assert t[k] == oracle.tau(s, int(pi[k]), int(pj[k]))
    with pytest.raises(oracle.OracleError):
        oracle.pair_timesteps(s, np.array([0], np.int32), np.array([n], np.int32))
