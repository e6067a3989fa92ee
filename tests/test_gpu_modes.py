"""GPU parity of the library's other modes through the C ABI: the plain path
(every set through the grid-wide kernels, no on-chip batching) and the
paper's softened 1024-body Plummer test (Sec. 3.1) under the CC and HOLD
splits, whose operation counts the paper prints."""
import numpy as np
import pytest

import oracle
import synth
from synth import Particles

from .gpu_util import assert_state_equal
from .golden import load_golden

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1407_7105_amd import CC_ORDER_EXACT, CC_ORDER_FAST, CCError, Context, State  # noqa: E402

STAT_KEYS = ("kick_pairs", "drifts", "components", "splits", "max_depth_seen")


def ctx_for(p: oracle.Params, **kw):
    kw.setdefault("kick_order", CC_ORDER_EXACT)
    return Context(device=0, eta=p.eta, eps2=p.eps2, G=p.G, max_depth=p.max_depth, hold=p.hold, **kw)


def run_both(s, dt, t_end, p, **kw):
    ref = s.copy()
    rc, ost = oracle.evolve(ref, dt, t_end, p)
    g = State.from_numpy(s)
    st = ctx_for(p, **kw).evolve(g, dt, t_end)
    return g.to_numpy(), ref, st, ost


# ------------------------------------------------------------------ plain path

@pytest.mark.parametrize("cfg,n", [(1, None), (2, 1500)])
def test_plain_one_step_bitwise(cfg, n):
    """Every component, two-body ones included, split and kicked by the
    grid-wide kernels one level visit at a time: bit-identical to the
    oracle with identical decisions."""
    s = synth.workload(cfg, n=n) if n else synth.workload(cfg)
    p = oracle.Params(eta=0.01)
    got, ref, st, ost = run_both(s, 1 / 64, 1 / 64, p, plain=1)
    assert_state_equal(got, ref, f"cfg{cfg}")
    for k in STAT_KEYS:
        assert st[k] == ost[k], (k, st[k], ost[k])


def test_plain_batch_and_hold_bitwise():
    """Independent clusters in one call, and the HOLD split, on the plain path."""
    sizes = [3, 40, 150, 90]
    parts = [synth.plummer(m, 700 + m, masses="salpeter") for m in sizes]
    # a cluster of two bodies: a circular pair whose step is below dt
    v = 0.5 * np.sqrt(0.5 / 0.05)
    parts.append(Particles.from_arrays(np.array([[0.0, 0.0, 0.0], [0.05, 0.0, 0.0]]),
                                       np.array([[0.0, -v, 0.0], [0.0, v, 0.0]]), np.array([0.25, 0.25])))
    sizes.append(2)
    s = Particles.from_arrays(np.concatenate([q.pos() for q in parts]), np.concatenate([q.vel() for q in parts]),
                              np.concatenate([q.m for q in parts]))
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    for hold in (0, 1):
        p = oracle.Params(eta=0.01, hold=hold)
        ref = s.copy()
        rc, osts = oracle.evolve_batch(ref, off, 1 / 64, 2 / 64, p)
        g = State.from_numpy(s)
        sts = ctx_for(p, plain=1).evolve_batch(g, off, 1 / 64, 2 / 64)
        assert_state_equal(g.to_numpy(), ref, f"hold={hold}")
        for c, (a, b) in enumerate(zip(sts, osts)):
            for k in STAT_KEYS:
                assert a[k] == b[k], (hold, c, k, a[k], b[k])


def test_plain_fast_order_matches_batched_decisions():
    """The benchmarked kick order on the plain path: one step of the
    1500-body Salpeter Plummer sphere agrees with the batched path to 1e-10
    relative and makes the same decisions."""
    s = synth.workload(2, n=1500)
    p = oracle.Params(eta=0.01)
    a, b = State.from_numpy(s), State.from_numpy(s)
    sa = ctx_for(p, kick_order=CC_ORDER_FAST, plain=1).evolve(a, 1 / 64, 1 / 64)
    sb = ctx_for(p, kick_order=CC_ORDER_FAST).evolve(b, 1 / 64, 1 / 64)
    for k in STAT_KEYS:
        assert sa[k] == sb[k], (k, sa[k], sb[k])
    ga, gb = a.to_numpy(), b.to_numpy()
    for f in ("x", "y", "z", "vx", "vy", "vz"):
        floor = 1e-6 * np.max(np.abs(gb[f]))
        err = np.abs(ga[f] - gb[f]) / np.maximum(np.abs(gb[f]), floor)
        assert err.max() <= 1e-10, (f, float(err.max()))


def test_plain_rejects_kepler():
    with pytest.raises(CCError) as e:
        Context(device=0, eta=0.01, plain=1, kepler=1)
    assert e.value.code == -1


# ------------------------------------------------------------------ the paper's softened Plummer test

@pytest.fixture(scope="module")
def paper():
    (rec,) = load_golden("paper_plummer1024_first_step.txt")
    return rec


@pytest.mark.parametrize("hold", [0, 1])
def test_paper_plummer1024_first_step_counts(paper, hold):
    """The first global step (dt = 700/512) of the softened 1024-body Plummer
    sphere: the GPU matches the oracle bit for bit with the same operation
    counts under both splits; the CC counts lie near the paper's."""
    s = synth.plummer(int(paper["n"]), 1)
    p = oracle.Params(eta=paper["eta"], eps2=paper["eps"] ** 2, hold=hold)
    got, ref, st, ost = run_both(s, paper["dt"], paper["dt"], p)
    assert_state_equal(got, ref, f"hold={hold}")
    for k in STAT_KEYS:
        assert st[k] == ost[k], (k, st[k], ost[k])
    if hold:
        assert st["tau_pairs_alg"] == ost["tau_evals"]
    else:
        assert st["tau_pairs_alg"] >= ost["tau_evals"]   # the BFS skips pairs of particles already placed
    if not hold:
        assert abs(ost["tau_evals"] / paper["tau_evals"] - 1) < 0.10
        assert abs(2 * st["kick_pairs"] / paper["kicks"] - 1) < 0.15
        assert abs(st["drifts"] / paper["drifts"] - 1) < 0.10
