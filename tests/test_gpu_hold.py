"""GPU parity of the HOLD split (Sec. 2.1, eqs. 11-17): the HIP library with
hold = 1 against the oracle's HOLD integrator, through the C ABI.

In the exact kick order every FP64 operation happens in the oracle's order,
so states are compared bit for bit, with the decisions (splits, components,
kicked pairs, drifts, depth) and the algorithmic pair-step count (HOLD needs
all n(n-1)/2 pair steps of every set it splits)."""
import math

import numpy as np
import pytest

import oracle
import synth
from synth import Particles

from .gpu_util import assert_state_equal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1407_7105_amd import CC_ORDER_EXACT, CC_ORDER_FAST, CCError, Context, State  # noqa: E402

STAT_KEYS = ("kick_pairs", "drifts", "components", "splits", "max_depth_seen")


def hold_ctx(p: oracle.Params, **kw):
    kw.setdefault("kick_order", CC_ORDER_EXACT)
    return Context(device=0, eta=p.eta, eps2=p.eps2, G=p.G, max_depth=p.max_depth, hold=1, **kw)


def run_both(s, dt, t_end, p, **kw):
    ref = s.copy()
    rc, ost = oracle.evolve(ref, dt, t_end, p)
    g = State.from_numpy(s)
    st = hold_ctx(p, **kw).evolve(g, dt, t_end)
    return g.to_numpy(), ref, st, ost


def check_stats(st, ost, what=""):
    for k in STAT_KEYS:
        assert st[k] == ost[k], (what, k, st[k], ost[k])
    assert st["tau_pairs_alg"] == ost["tau_evals"], (what, st["tau_pairs_alg"], ost["tau_evals"])


@pytest.mark.parametrize("small_max", [0, 16, 3])
def test_hold_plummer256_one_step_bitwise(small_max):
    """The 256-body Plummer sphere: on chip (default limit), on the grid
    below 17 bodies, and with every set of three or more on the grid."""
    s = synth.workload(1)
    p = oracle.Params(eta=0.01, hold=1)
    got, ref, st, ost = run_both(s, 1 / 64, 1 / 64, p, small_max=small_max)
    assert ost["components"] > 0
    assert_state_equal(got, ref, f"small_max={small_max}")
    check_stats(st, ost, f"small_max={small_max}")


def test_hold_plummer256_to_t1_bitwise():
    s = synth.workload(1)
    p = oracle.Params(eta=0.01, hold=1)
    got, ref, st, ost = run_both(s, 1 / 64, 1.0, p)
    assert_state_equal(got, ref, "t=1")
    check_stats(st, ost, "t=1")


@pytest.mark.parametrize("n,small_max", [(1500, 0), (1500, 64), (3000, 256)])
def test_hold_grid_path_bitwise(n, small_max):
    """Sets above the on-chip limit: the grid path merges the components of
    each segment into F (labels and sort keys) before the sort."""
    s = synth.plummer(n, 77 + n, masses="salpeter")
    p = oracle.Params(eta=0.01, hold=1)
    got, ref, st, ost = run_both(s, 1 / 64, 1 / 64, p, small_max=small_max)
    assert_state_equal(got, ref, f"n={n}")
    check_stats(st, ost, f"n={n}")


@pytest.mark.parametrize("sizes,small_max", [([3, 40, 150, 700, 20, 300], 128), ([12, 31, 5, 64], 0)])
def test_hold_batch_bitwise(sizes, small_max):
    """Independent Plummer clusters in one batch: F is formed per cluster
    (per segment on the grid path, per set on chip), never across clusters."""
    parts = [synth.plummer(m, 900 + m, masses="salpeter") for m in sizes]
    s = Particles.from_arrays(np.concatenate([q.pos() for q in parts]), np.concatenate([q.vel() for q in parts]),
                              np.concatenate([q.m for q in parts]))
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    p = oracle.Params(eta=0.01, hold=1)
    ref = s.copy()
    rc, osts = oracle.evolve_batch(ref, off, 1 / 64, 2 / 64, p)
    g = State.from_numpy(s)
    sts = hold_ctx(p, small_max=small_max).evolve_batch(g, off, 1 / 64, 2 / 64)
    assert_state_equal(g.to_numpy(), ref, "batch")
    for c, (a, b) in enumerate(zip(sts, osts)):
        check_stats(a, b, f"cluster {c}")


def circular_binaries(K, a, spacing, mass=1.0, seed=3):
    rng = np.random.default_rng(seed)
    pos, vel = [], []
    v = math.sqrt(mass / a) / 2.0
    for k in range(K):
        c = np.array([k * spacing, 0.0, 0.0])
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        w = np.cross(d, rng.normal(size=3))
        w /= np.linalg.norm(w)
        pos += [c - 0.5 * a * d, c + 0.5 * a * d]
        vel += [-v * w, v * w]
    return Particles.from_arrays(np.array(pos), np.array(vel), np.full(2 * K, mass / 2.0))


@pytest.mark.parametrize("K", [5, 40])
def test_hold_isolated_binaries_share_one_step(K):
    """K isolated binaries whose pair step lies between dt0/16 and dt0/8: the
    CC split integrates each binary alone, HOLD keeps all 2K bodies in F down
    to depth 4, so every pair is kicked 16 times (Sec. 2.1).  40 binaries
    (80 bodies) are split on chip, 5 binaries with an on-chip limit of 3 on
    the grid path."""
    mass, dt, L, eta = 1.0, 1 / 64, 4, 0.01
    a = (0.75 * dt / 2 ** (L - 1) * math.sqrt(mass) / eta) ** (2 / 3)
    s = circular_binaries(K, a, spacing=50.0, mass=mass)
    n = 2 * K
    p = oracle.Params(eta=eta, hold=1)
    got, ref, st, ost = run_both(s, dt, dt, p, small_max=3 if K == 5 else 0)
    assert_state_equal(got, ref, f"K={K}")
    check_stats(st, ost, f"K={K}")
    assert st["kick_pairs"] == 2 ** L * n * (n - 1) // 2 and st["max_depth_seen"] == L


def test_hold_star_levels_on_grid_and_on_chip():
    """A set whose first levels are fully connected (stars): under HOLD the
    whole set is F, split again at h/2; the grid path (on-chip limit 64) and
    the on-chip split (limit 128) both match the oracle bit for bit."""
    n = 300
    rng = np.random.default_rng(21)
    pos = rng.normal(size=(n, 3)) * rng.uniform(0.01, 1.0, (n, 1))
    s = Particles.from_arrays(pos, rng.normal(size=(n, 3)), rng.uniform(0.1, 1.0, n) / n)
    p = oracle.Params(eta=0.01, hold=1)
    i, j = np.triu_indices(n, 1)
    tau = oracle.pair_timesteps(s, i.astype(np.int32), j.astype(np.int32), p)
    dt = 2.5 * float(tau.max())
    ref = s.copy()
    rc, ost = oracle.evolve(ref, dt, 2 * dt, p)
    for small_max in (64, 128):
        g = State.from_numpy(s)
        st = hold_ctx(p, small_max=small_max).evolve(g, dt, 2 * dt)
        assert_state_equal(g.to_numpy(), ref, f"small_max={small_max}")
        check_stats(st, ost, f"small_max={small_max}")


@pytest.mark.parametrize("cfg,n,small_max", [(1, None, 0), (2, 1500, 64)])
def test_hold_fast_order_one_step_lockstep(cfg, n, small_max):
    """The fast kick order under HOLD: one global step agrees with the oracle
    to 1e-10 relative per particle and makes the same decisions."""
    s = synth.workload(cfg, n=n) if n else synth.workload(cfg)
    p = oracle.Params(eta=0.01, hold=1)
    ref = s.copy()
    rc, ost = oracle.evolve(ref, 1 / 64, 1 / 64, p)
    g = State.from_numpy(s)
    st = hold_ctx(p, kick_order=CC_ORDER_FAST, small_max=small_max).evolve(g, 1 / 64, 1 / 64)
    got = g.to_numpy()
    for f in ("x", "y", "z", "vx", "vy", "vz"):
        a, b = got[f], getattr(ref, f)
        floor = 1e-6 * np.max(np.abs(b))
        err = np.abs(a - b) / np.maximum(np.abs(b), floor)
        assert err.max() <= 1e-10, (f, float(err.max()))
    check_stats(st, ost, f"cfg{cfg}")


def test_hold_with_kepler_is_rejected():
    with pytest.raises(CCError) as e:
        Context(device=0, eta=0.01, hold=1, kepler=1)
    assert e.value.code == -1
    with pytest.raises(CCError):
        Context(device=0, eta=0.01, hold=2)
