"""Seeded synthetic initial conditions for the CC integrator workloads.

This module only generates inputs (positions, velocities, masses).  It holds
none of the integrator's arithmetic and is shared by the oracle tests, the GPU
tests and the benchmark, so that both sides see identical inputs.

All generators use numpy's PCG64 with an explicit seed and return a
:class:`Particles` record of float64 arrays in N-body (Henon) units
(G = 1, total mass 1, E = -1/4 for the cluster before binaries are inserted).

Published methods used (written here from their descriptions):
  * Plummer sphere sampling: Aarseth, Henon & Wielen (1974).
  * Salpeter mass function dN/dm ~ m^-2.35 by inverse-CDF sampling.
  * Box fractal: Goodwin & Whitworth (2004) -- cube subdivision with child
    survival probability 2^(D-3).
  * Binaries: Keplerian two-body orbits with log-uniform semi-major axis,
    thermal eccentricity, isotropic orientation and uniform mean anomaly.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 14077105

__all__ = [
    "Particles", "plummer", "salpeter", "fractal", "with_binaries", "cluster_ensemble",
    "workload", "WORKLOADS", "henon_scale", "random_pairs",
]


@dataclass
class Particles:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    m: np.ndarray
    offsets: np.ndarray | None = None   # cluster boundaries for ensembles
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.m.shape[0])

    def arrays(self):
        return (self.x, self.y, self.z, self.vx, self.vy, self.vz, self.m)

    def copy(self) -> "Particles":
        return Particles(*(a.copy() for a in self.arrays()),
                         offsets=None if self.offsets is None else self.offsets.copy(),
                         meta=dict(self.meta))

    @staticmethod
    def from_arrays(pos: np.ndarray, vel: np.ndarray, m: np.ndarray, **meta) -> "Particles":
        pos = np.asarray(pos, dtype=np.float64)
        vel = np.asarray(vel, dtype=np.float64)
        m = np.ascontiguousarray(m, dtype=np.float64)
        return Particles(np.ascontiguousarray(pos[:, 0]), np.ascontiguousarray(pos[:, 1]),
                         np.ascontiguousarray(pos[:, 2]), np.ascontiguousarray(vel[:, 0]),
                         np.ascontiguousarray(vel[:, 1]), np.ascontiguousarray(vel[:, 2]), m,
                         meta=dict(meta))

    def pos(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)

    def vel(self) -> np.ndarray:
        return np.stack([self.vx, self.vy, self.vz], axis=1)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    cz = 1.0 - 2.0 * rng.random(n)
    ph = 2.0 * np.pi * rng.random(n)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return np.stack([sz * np.cos(ph), sz * np.sin(ph), cz], axis=1)


def salpeter(n: int, rng: np.random.Generator, mmin: float = 0.1, mmax: float = 100.0,
             alpha: float = 2.35) -> np.ndarray:
    """Masses from dN/dm ~ m^-alpha on [mmin, mmax] (inverse CDF), unnormalised."""
    e = 1.0 - alpha
    u = rng.random(n)
    return (mmin ** e + u * (mmax ** e - mmin ** e)) ** (1.0 / e)


def _potential(pos: np.ndarray, m: np.ndarray, chunk: int = 512) -> float:
    """Exact potential energy sum_{i<j} -m_i m_j / r_ij (G = 1), chunked."""
    n = len(m)
    w = 0.0
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        d = pos[a:b, None, :] - pos[None, :, :]
        r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
        idx_i = np.arange(a, b)[:, None]
        idx_j = np.arange(n)[None, :]
        mask = idx_j > idx_i
        with np.errstate(divide="ignore"):
            w -= float(np.sum(np.where(mask, (m[a:b, None] * m[None, :]) / np.where(mask, r, 1.0), 0.0)))
    return w


EXACT_SCALE_MAX_N = 20000


def henon_scale(pos: np.ndarray, vel: np.ndarray, m: np.ndarray, q_vir: float = 0.5,
                exact: bool | None = None):
    """Shift to the centre-of-mass frame and scale to E = -1/4, T/|W| = q_vir.

    For n <= EXACT_SCALE_MAX_N the potential is summed exactly; larger sets are
    assumed to be already in model units with virial radius 1 (the expected
    potential of such a set is -1/2) and only the kinetic energy is rescaled.
    With all velocities zero (cold start) only the positions are scaled.
    """
    m = m / m.sum()
    pos = pos - (m[:, None] * pos).sum(0)
    vel = vel - (m[:, None] * vel).sum(0)
    n = len(m)
    if exact is None:
        exact = n <= EXACT_SCALE_MAX_N
    t = 0.5 * float(np.sum(m * np.sum(vel * vel, axis=1)))
    if exact:
        w = _potential(pos, m)
    else:
        w = -0.5
    if t > 0.0:
        # want T' = q |W'| and T' + W' = -1/4  ->  W' = -1/(4 (1 - q)), T' = -q W'
        w_target = -0.25 / (1.0 - q_vir)
        t_target = -q_vir * w_target
        pos = pos * (w / w_target)
        vel = vel * np.sqrt(t_target / t)
    else:
        pos = pos * (w / -0.25)
    return pos, vel, m


def _masses(masses, n: int, rng: np.random.Generator) -> np.ndarray:
    if isinstance(masses, np.ndarray):
        assert masses.shape == (n,)
        return masses.astype(np.float64)
    if masses == "equal":
        return np.full(n, 1.0 / n)
    if masses == "salpeter":
        return salpeter(n, rng)
    raise ValueError(masses)


def plummer(n: int, seed: int, masses="equal", q_vir: float = 0.5) -> Particles:
    """Plummer sphere in Henon units (Aarseth, Henon & Wielen 1974)."""
    rng = _rng(seed)
    x1 = rng.random(n) * 0.999
    x1 = np.maximum(x1, 1e-300)
    r = 1.0 / np.sqrt(x1 ** (-2.0 / 3.0) - 1.0)
    pos = r[:, None] * _isotropic(rng, n)
    q = np.empty(n)
    k = 0
    while k < n:
        cand = rng.random(2 * (n - k) + 16)
        ys = rng.random(cand.shape[0]) * 0.1
        ok = cand[ys < cand * cand * (1.0 - cand * cand) ** 3.5]
        take = min(n - k, ok.shape[0])
        q[k:k + take] = ok[:take]
        k += take
    speed = q * np.sqrt(2.0) * (1.0 + r * r) ** -0.25
    vel = speed[:, None] * _isotropic(rng, n)
    m = _masses(masses, n, rng)
    # Plummer model units -> virial radius 1 before the (exact) rescale
    pos = pos * (3.0 * np.pi / 16.0)
    vel = vel * np.sqrt(16.0 / (3.0 * np.pi))
    pos, vel, m = henon_scale(pos, vel, m, q_vir)
    return Particles.from_arrays(pos, vel, m, kind="plummer", n=n, seed=seed, masses=masses)


def fractal(n: int, seed: int, dim: float = 1.6, q_vir: float = 0.5, cold: bool = False,
            masses="equal") -> Particles:
    """Goodwin & Whitworth (2004) box fractal of dimension dim in Henon units."""
    rng = _rng(seed)
    p_keep = 2.0 ** (dim - 3.0)
    while True:
        pos = np.zeros((1, 3))
        vel = np.zeros((1, 3))
        side = 2.0
        gen = 0
        while True:
            gen += 1
            side *= 0.5
            offs = np.array([[sx, sy, sz] for sx in (-0.5, 0.5) for sy in (-0.5, 0.5)
                             for sz in (-0.5, 0.5)]) * side
            cpos = (pos[:, None, :] + offs[None, :, :]).reshape(-1, 3)
            cvel = np.repeat(vel, 8, axis=0) + rng.standard_normal((cpos.shape[0], 3)) * 2.0 ** (-gen)
            keep = rng.random(cpos.shape[0]) < p_keep
            pos, vel = cpos[keep], cvel[keep]
            if pos.shape[0] == 0:
                break
            inside = np.sum(pos * pos, axis=1) < 1.0
            if inside.sum() > n:
                break
        if pos.shape[0] == 0:
            continue
        pos = pos + (rng.random(pos.shape) - 0.5) * 0.5 * side
        inside = np.sum(pos * pos, axis=1) < 1.0
        if inside.sum() < n:
            continue
        idx = np.flatnonzero(inside)
        pick = np.sort(rng.choice(idx, size=n, replace=False))
        pos, vel = pos[pick], vel[pick]
        break
    m = _masses(masses, n, rng)
    if cold:
        vel = np.zeros_like(vel)
    pos, vel, m = henon_scale(pos, vel, m, q_vir, exact=n <= EXACT_SCALE_MAX_N if not cold else None)
    return Particles.from_arrays(pos, vel, m, kind="fractal", n=n, seed=seed, dim=dim)


def _kepler_E(M: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Solve Kepler's equation E - e sin E = M by Newton iteration."""
    E = np.where(e < 0.8, M, np.pi * np.ones_like(M))
    for _ in range(60):
        f = E - e * np.sin(E) - M
        E = E - f / (1.0 - e * np.cos(E))
    return E


def _random_rotation(rng: np.random.Generator, k: int) -> np.ndarray:
    q = rng.standard_normal((k, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((k, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z); R[:, 0, 1] = 2 * (x * y - z * w); R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w); R[:, 1, 1] = 1 - 2 * (x * x + z * z); R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w); R[:, 2, 1] = 2 * (y * z + x * w); R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def with_binaries(base: Particles, chosen: np.ndarray, loga: tuple[float, float], seed: int,
                  equal_mass: bool = True, emax: float = 0.999) -> Particles:
    """Replace the systems `chosen` of `base` by Keplerian binaries.

    Each binary keeps its system's centre-of-mass position, velocity and mass.
    Component masses are equal halves or split by two Salpeter draws; the
    semi-major axis is log-uniform in 10**loga, the eccentricity thermal
    (e = sqrt(U), redrawn above emax), the orientation isotropic and the mean
    anomaly uniform.  The two members of a binary get neighbouring indices.
    """
    rng = _rng(seed)
    chosen = np.sort(np.asarray(chosen, dtype=np.int64))
    nsys = base.n
    nbin = chosen.shape[0]
    single = np.ones(nsys, bool)
    single[chosen] = False
    pos, vel, m = base.pos(), base.vel(), base.m
    M = m[chosen]
    if equal_mass:
        q = np.full(nbin, 0.5)
    else:
        a1, a2 = salpeter(nbin, rng), salpeter(nbin, rng)
        q = a1 / (a1 + a2)
    m1, m2 = M * q, M * (1.0 - q)
    a = 10.0 ** rng.uniform(loga[0], loga[1], nbin)
    e = np.sqrt(rng.random(nbin))
    bad = e > emax
    while np.any(bad):
        e[bad] = np.sqrt(rng.random(int(bad.sum())))
        bad = e > emax
    Mmean = rng.uniform(0.0, 2.0 * np.pi, nbin)
    E = _kepler_E(Mmean, e)
    mu = M  # G = 1
    rel_r = np.stack([a * (np.cos(E) - e), a * np.sqrt(1 - e * e) * np.sin(E), np.zeros(nbin)], 1)
    fac = np.sqrt(mu / a) / (1.0 - e * np.cos(E))
    rel_v = np.stack([-fac * np.sin(E), fac * np.sqrt(1 - e * e) * np.cos(E), np.zeros(nbin)], 1)
    R = _random_rotation(rng, nbin)
    rel_r = np.einsum("kij,kj->ki", R, rel_r)
    rel_v = np.einsum("kij,kj->ki", R, rel_v)
    p1 = pos[chosen] - (m2 / M)[:, None] * rel_r
    p2 = pos[chosen] + (m1 / M)[:, None] * rel_r
    v1 = vel[chosen] - (m2 / M)[:, None] * rel_v
    v2 = vel[chosen] + (m1 / M)[:, None] * rel_v
    P = np.concatenate([pos[single], p1, p2])
    V = np.concatenate([vel[single], v1, v2])
    Mm = np.concatenate([m[single], m1, m2])
    # interleave so each binary's two members are neighbours in index order
    ns = int(single.sum())
    order = np.concatenate([np.arange(ns), np.stack([ns + np.arange(nbin), ns + nbin + np.arange(nbin)], 1).ravel()])
    out = Particles.from_arrays(P[order], V[order], Mm[order], **base.meta)
    out.meta.update(binaries=nbin, loga=tuple(loga))
    return out


def _n_systems(n: int, frac: float) -> tuple[int, int]:
    nbin = int(round(frac * n / (1.0 + frac)))
    return n - nbin, nbin


def cluster_ensemble(ncl: int, nmin: int, nmax: int, frac: float, loga: tuple[float, float],
                     seed: int) -> Particles:
    """ncl independent Plummer clusters with N_k ~ U{nmin..nmax}; offsets mark them."""
    rng = _rng(seed)
    sizes = rng.integers(nmin, nmax + 1, size=ncl)
    parts = []
    for k, nk in enumerate(sizes):
        nsys, nbin = _n_systems(int(nk), frac)
        ks = seed + 1000 * (k + 1)
        chosen, w = _binary_systems(nsys, nbin, ks + 7)
        base = plummer(nsys, ks, masses=w / w.sum())
        p = with_binaries(base, chosen, loga, ks + 11, equal_mass=True) if nbin else base
        parts.append(p)
    off = np.zeros(ncl + 1, np.int64)
    off[1:] = np.cumsum([p.n for p in parts])
    cat = [np.concatenate([getattr(p, f) for p in parts]) for f in ("x", "y", "z", "vx", "vy", "vz", "m")]
    out = Particles(*cat, offsets=off, meta=dict(kind="ensemble", ncl=ncl, seed=seed))
    return out


def _binary_systems(nsys: int, nbin: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Pick the nbin systems that become binaries; equal-mass stars give those
    systems twice the mass of a single star (weights before normalisation)."""
    rng = _rng(seed)
    chosen = np.sort(rng.choice(nsys, size=nbin, replace=False)) if nbin else np.zeros(0, np.int64)
    w = np.ones(nsys)
    w[chosen] = 2.0
    return chosen, w


def random_pairs(n: int, npairs: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    rng = _rng(seed)
    i = rng.integers(0, n, size=npairs).astype(np.int32)
    j = rng.integers(0, n - 1, size=npairs).astype(np.int32)
    j = np.where(j >= i, j + 1, j).astype(np.int32)
    return i, j


# ---------------------------------------------------------------------------
# The five workloads (sizes and physics parameters of the measured configurations)
# ---------------------------------------------------------------------------

WORKLOADS = {
    1: dict(name="plummer256_equal", n=256, eta=0.01, eps2=0.0, dt=1.0 / 64, t_end=1.0),
    2: dict(name="plummer16k_salpeter", n=16384, eta=0.01, eps2=0.0, dt=1.0 / 64, t_end=1.0 / 64),
    3: dict(name="fractal64k_d1.6_bin30", n=65536, eta=0.01, eps2=0.0, dt=1.0 / 64, t_end=1.0 / 8),
    4: dict(name="ensemble1024_plummer16-512_bin20", n=None, eta=0.01, eps2=0.0, dt=1.0 / 64, t_end=1.0),
    5: dict(name="plummer256k_salpeter_bin10", n=262144, eta=0.01, eps2=0.0, dt=1.0 / 64, t_end=1.0 / 16),
}


def workload(cfg: int, n: int | None = None) -> Particles:
    """Initial conditions of workload `cfg` (optionally at a smaller size n)."""
    seed = BASE_SEED + cfg
    if cfg == 1:
        return plummer(n or 256, seed, masses="equal")
    if cfg == 2:
        return plummer(n or 16384, seed, masses="salpeter")
    if cfg == 3:
        N = n or 65536
        nsys, nbin = _n_systems(N, 0.3)
        chosen, w = _binary_systems(nsys, nbin, seed + 7)
        base = fractal(nsys, seed, dim=1.6, masses=w / w.sum())
        return with_binaries(base, chosen, (-4.0, -1.0), seed + 11, equal_mass=True)
    if cfg == 4:
        if n is not None:
            return cluster_ensemble(n, 16, 64, 0.2, (-4.0, -1.0), seed)
        return cluster_ensemble(1024, 16, 512, 0.2, (-4.0, -1.0), seed)
    if cfg == 5:
        N = n or 262144
        nsys, nbin = _n_systems(N, 0.1)
        chosen, _ = _binary_systems(nsys, nbin, seed + 7)
        base = plummer(nsys, seed, masses="salpeter")
        return with_binaries(base, chosen, (-5.0, -3.0), seed + 11, equal_mass=False)
    raise ValueError(cfg)
