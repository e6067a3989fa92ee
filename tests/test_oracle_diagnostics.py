"""Pins of the oracle's integrals of motion (eqs. 1-3): kinetic and potential
energy, linear and angular momentum, centre of mass and total mass, checked
against closed forms that do not go through the oracle's own sums.

Every one of the twelve outputs is compared with an absolute value, so a sign
or factor error in any of them (a flipped potential, a missing 1/2, a swapped
cross-product component, a COM not divided by the mass) fails a test here."""
import math

import numpy as np
import pytest

import oracle
import synth
from synth import Particles


def kepler_pair(m1, m2, a, e, G=1.0, X0=(0.0, 0.0, 0.0), V0=(0.0, 0.0, 0.0)):
    """Two bodies at pericentre of a Kepler orbit (semi-major axis a,
    eccentricity e) in the x-y plane, the pair's centre of mass at X0 moving
    with V0.  Returns the state and the closed-form integrals."""
    M = m1 + m2
    rp = a * (1.0 - e)
    vp = math.sqrt(G * M * (1.0 + e) / (a * (1.0 - e)))
    X0 = np.asarray(X0, float)
    V0 = np.asarray(V0, float)
    pos = np.array([[-m2 / M * rp, 0.0, 0.0], [m1 / M * rp, 0.0, 0.0]]) + X0
    vel = np.array([[0.0, -m2 / M * vp, 0.0], [0.0, m1 / M * vp, 0.0]]) + V0
    s = Particles.from_arrays(pos, vel, np.array([m1, m2]))
    mu_red = m1 * m2 / M
    # closed forms: E_int = -G m1 m2 / (2a); |L_int| = mu_red sqrt(G M a (1 - e^2))
    want = dict(
        epot=-G * m1 * m2 / rp,
        ekin=0.5 * M * float(V0 @ V0) + 0.5 * mu_red * vp * vp,
        E_int=-G * m1 * m2 / (2.0 * a),
        P=M * V0,
        L=np.array([0.0, 0.0, mu_red * math.sqrt(G * M * a * (1.0 - e * e))]) + M * np.cross(X0, V0),
        com=X0,
        mass=M,
    )
    return s, want


@pytest.mark.parametrize("e", [0.0, 0.5, 0.9])
@pytest.mark.parametrize("G", [1.0, 0.75])
def test_kepler_pair_integrals_closed_form(e, G):
    m1, m2, a = 0.3, 0.5, 0.04
    s, w = kepler_pair(m1, m2, a, e, G=G)
    d = oracle.diagnostics(s, oracle.Params(G=G))
    # internal energy of a bound pair: -G m1 m2 / (2a) (vis-viva)
    assert d["energy"] == pytest.approx(w["E_int"], rel=1e-14)
    assert d["epot"] == pytest.approx(w["epot"], rel=1e-14)
    assert d["ekin"] == pytest.approx(w["ekin"], rel=1e-14)
    assert np.allclose(d["L"], w["L"], rtol=1e-14, atol=1e-16)
    # zero up to the rounding of the input construction
    pscale = float(np.sum(s.m * np.linalg.norm(s.vel(), axis=1)))
    xscale = float(np.sum(s.m * np.linalg.norm(s.pos(), axis=1))) / (m1 + m2)
    assert np.all(np.abs(d["P"]) <= 4e-16 * pscale)
    assert np.all(np.abs(d["com"]) <= 4e-16 * xscale)
    assert d["mass"] == m1 + m2


def test_kepler_pair_in_a_moving_frame():
    """The same pair displaced and boosted: P = M V0, COM = X0,
    L = L_int + M X0 x V0, T = T_int + M V0^2 / 2, W unchanged."""
    X0, V0 = (0.25, -1.5, 2.0), (0.125, 0.5, -0.75)
    s, w = kepler_pair(0.2, 0.6, 0.01, 0.5, X0=X0, V0=V0)
    d = oracle.diagnostics(s)
    assert d["epot"] == pytest.approx(w["epot"], rel=1e-14)
    assert d["ekin"] == pytest.approx(w["ekin"], rel=1e-13)
    assert np.allclose(d["P"], w["P"], rtol=1e-15, atol=0)
    assert np.allclose(d["com"], w["com"], rtol=1e-15, atol=1e-17)
    assert np.allclose(d["L"], w["L"], rtol=1e-13, atol=1e-16)
    assert d["mass"] == pytest.approx(0.8, rel=1e-16)


def test_softened_potential_closed_form():
    """V_ij = -G m_i m_j / sqrt(r^2 + eps^2) (eq. 3): r = 3, eps = 4 gives 5."""
    s = Particles.from_arrays(np.array([[0.0, 0, 0], [3.0, 0, 0]]), np.zeros((2, 3)), np.array([2.0, 5.0]))
    d = oracle.diagnostics(s, oracle.Params(eps2=16.0, G=2.0))
    assert d["epot"] == -2.0 * 2.0 * 5.0 / 5.0
    assert d["ekin"] == 0.0


def test_hand_built_three_body_exact():
    """Three bodies with small integer coordinates: every output is exact in
    binary floating point, so it is compared for equality."""
    pos = np.array([[1.0, 0.0, 0.0], [0.0, 2.0, 0.0], [0.0, 0.0, 4.0]])
    vel = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, -1.0], [2.0, 0.0, 0.0]])
    m = np.array([1.0, 2.0, 0.5])
    s = Particles.from_arrays(pos, vel, m)
    d = oracle.diagnostics(s)
    # T = 1/2 (1*1 + 2*1 + 0.5*4) = 2.5
    assert d["ekin"] == 2.5
    # P = (0.5*2, 1*1, 2*(-1)) = (1, 1, -2)
    assert np.array_equal(d["P"], [1.0, 1.0, -2.0])
    # L = sum m r x v: 1*(0,0,1) + 2*(-2,0,0) + 0.5*(0,8,0) = (-4, 4, 1)
    assert np.array_equal(d["L"], [-4.0, 4.0, 1.0])
    # COM = (1, 4, 2) / 3.5
    assert np.allclose(d["com"], np.array([1.0, 4.0, 2.0]) / 3.5, rtol=1e-16, atol=0)
    assert d["mass"] == 3.5
    # W = -(1*2/sqrt5 + 1*0.5/sqrt17 + 2*0.5/sqrt20)
    w = -(2.0 / math.sqrt(5.0) + 0.5 / math.sqrt(17.0) + 1.0 / math.sqrt(20.0))
    assert d["epot"] == pytest.approx(w, rel=1e-15)


@pytest.mark.parametrize("seed", [1, 2])
def test_plummer_generator_energy_and_virial_ratio(seed):
    """The generator scales a Plummer sphere to E = -1/4 and T/|W| = 1/2 with
    its own potential sum; the oracle's compensated sums must agree."""
    p = synth.plummer(1000, seed)
    d = oracle.diagnostics(p)
    assert d["energy"] == pytest.approx(-0.25, rel=1e-12)
    assert d["ekin"] / -d["epot"] == pytest.approx(0.5, rel=1e-12)
    assert d["mass"] == pytest.approx(1.0, rel=1e-14)
    assert np.all(np.abs(d["P"]) < 1e-15) and np.all(np.abs(d["com"]) < 1e-15)
