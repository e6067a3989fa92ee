"""The GPU's two-body flow (CC_KEPLER), built for the host from the same
header the kernels include, on the CPU: against the classical anomaly
solution (mpmath, 40 digits) and against the oracle's independent
universal-variable solver on random conics -- bound, near-parabolic and
hyperbolic, forwards and backwards, over up to thousands of periods."""
import ctypes as C
import math
import os
import subprocess

import numpy as np
import pytest

import oracle

from .test_oracle_kepler import classical_state, mean_motion

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def flow(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("kepler") / "libkepler.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    os.path.join(HERE, "kepler_shim.cpp"), "-o", out], check=True)
    lib = C.CDLL(out)
    lib.kepler_flow_host.restype = C.c_int
    lib.kepler_flow_host.argtypes = [C.c_double, C.POINTER(C.c_double), C.c_double]

    def f(mu, r, v, t):
        rv = np.ascontiguousarray(np.concatenate([np.asarray(r, float), np.asarray(v, float)]))
        assert lib.kepler_flow_host(mu, rv.ctypes.data_as(C.POINTER(C.c_double)), t) == 1
        return rv[:3], rv[3:]
    return f


@pytest.mark.parametrize("e", [0.0, 0.5, 0.9, 0.999])
@pytest.mark.parametrize("M0,periods", [(0.3, 0.37), (2.5, -1.0), (0.0, 12.25), (5.9, -101.6)])
def test_device_flow_elliptic_against_anomaly_solution(flow, e, M0, periods):
    mu, a = 0.7, 0.013
    n = mean_motion(mu, a)
    dt = periods * 2 * math.pi / n
    r0, v0 = classical_state(mu, a, e, M0)
    r, v = flow(mu, r0, v0, dt)
    rw, vw = classical_state(mu, a, e, M0 + n * dt)
    tol = 1e-13 * (1 + abs(periods))
    assert np.max(np.abs(r - rw)) <= tol * a * (1 + e) / max(1 - e, 1e-3)
    assert np.max(np.abs(v - vw)) <= tol * math.sqrt(mu / a) * math.sqrt((1 + e) / (1 - e)) / max(1 - e, 1e-3)


@pytest.mark.parametrize("e", [1.2, 3.0])
@pytest.mark.parametrize("M0,dM", [(0.0, 0.5), (-4.0, 6.0), (1.0, 40.0), (3.0, -20.0)])
def test_device_flow_hyperbolic_against_anomaly_solution(flow, e, M0, dM):
    mu, a = 1.3, 0.05
    n = mean_motion(mu, a)
    r0, v0 = classical_state(mu, a, e, M0)
    r, v = flow(mu, r0, v0, dM / n)
    rw, vw = classical_state(mu, a, e, M0 + dM)
    assert np.max(np.abs(r - rw)) <= 1e-12 * np.linalg.norm(rw)
    assert np.max(np.abs(v - vw)) <= 1e-12 * max(np.linalg.norm(vw), math.sqrt(mu / a))


def _random_conic(rng, kind):
    mu = 10.0 ** rng.uniform(-7, 0)
    a = 10.0 ** rng.uniform(-6, -1)
    e = [rng.uniform(0, 0.9), 1 - 10.0 ** rng.uniform(-4, -1), rng.uniform(1.01, 5)][kind]
    if e < 1:
        nu, p = rng.uniform(-np.pi, np.pi), a * (1 - e * e)
    else:
        nu, p = rng.uniform(-1, 1) * np.arccos(-1 / e) * 0.99, a * (e * e - 1)
    r = p / (1 + e * np.cos(nu))
    rvec = np.array([r * np.cos(nu), r * np.sin(nu), 0.0])
    vvec = np.sqrt(mu / p) * np.array([-np.sin(nu), e + np.cos(nu), 0.0])
    P = 2 * np.pi * np.sqrt(a ** 3 / mu)
    return mu, rvec, vvec, P * 10.0 ** rng.uniform(-3, 3.5) * rng.choice([1, -1])


@pytest.mark.parametrize("kind,tol", [(0, 1e-12), (1, 1e-8), (2, 1e-11)])
def test_device_flow_against_oracle_solver(flow, kind, tol):
    """Bound (e < 0.9), near-parabolic (1 - e down to 1e-4) and hyperbolic
    conics at random phases and times: the two codes agree to their
    conditioning."""
    rng = np.random.default_rng(100 + kind)
    for _ in range(3000):
        mu, r0, v0, t = _random_conic(rng, kind)
        ro, vo = oracle.kepler(mu, r0, v0, t)
        rd, vd = flow(mu, r0, v0, t)
        assert np.linalg.norm(rd - ro) <= tol * np.linalg.norm(ro), (mu, r0, v0, t)
        assert np.linalg.norm(vd - vo) <= tol * np.linalg.norm(vo), (mu, r0, v0, t)
