"""cc_kick_static, the kick that allocates nothing (scratch in a static device
array of the library), against cc_kick through the C ABI: bit-identical
results on two calls in a row, the second one smaller; sizes beyond the limit
rejected; an error call does not leak its flag into the next call."""
import numpy as np
import pytest

import synth
from synth import Particles

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1407_7105_amd import CC_FP64, CC_MIXED, CCError, Context, State  # noqa: E402
from paper_1407_7105_amd.cc import KICK_STATIC_MAX_N  # noqa: E402


def _both(ctx, p, h, label=None):
    a, b = State.from_numpy(p), State.from_numpy(p)
    lab = None if label is None else torch.from_numpy(label)
    ctx.kick(a, h, lab)
    ctx.kick_static(b, h, lab)
    return a.to_numpy(), b.to_numpy()


@pytest.mark.parametrize("precision", [CC_FP64, CC_MIXED])
def test_kick_static_equals_kick_on_two_calls(precision):
    print(f"\n# cc_kick_static vs cc_kick, precision {precision}: n = {KICK_STATIC_MAX_N} then 3001", flush=True)
    ctx = Context(device=0, eta=0.01, eps2=1e-6, precision=precision)
    big = synth.plummer(KICK_STATIC_MAX_N, 3, masses="salpeter")   # the largest size allowed
    small = synth.plummer(3001, 4)
    lab = np.random.default_rng(5).integers(0, 9, small.n).astype(np.int32)
    for p, label in ((big, None), (small, lab)):
        a, b = _both(ctx, p, 0.01, label)
        for f in State.FIELDS:
            assert np.array_equal(a[f], b[f]), (p.n, f)
        assert not np.array_equal(a["vx"], p.vx)   # the kick did something
    ctx.close()


def test_kick_static_rejects_beyond_limit_and_clears_errors():
    ctx = Context(device=0, eta=0.01, eps2=0.0)
    p = synth.plummer(KICK_STATIC_MAX_N + 1, 6)
    g = State.from_numpy(p)
    with pytest.raises(CCError) as e:
        ctx.kick_static(g, 0.01)
    assert e.value.code == -1
    assert np.array_equal(g.to_numpy()["vx"], p.vx)
    # a coincident pair: the error flag is raised and the state left alone ...
    bad = synth.plummer(100, 7)
    bad.x[5], bad.y[5], bad.z[5] = bad.x[9], bad.y[9], bad.z[9]
    g = State.from_numpy(bad)
    with pytest.raises(CCError) as e:
        ctx.kick_static(g, 0.01)
    assert e.value.code == -2
    assert np.array_equal(g.to_numpy()["vx"], bad.vx)
    # ... and the next call starts from a clear flag
    ok = synth.plummer(100, 8)
    a, b = _both(ctx, ok, 0.01)
    for f in State.FIELDS:
        assert np.array_equal(a[f], b[f]), f
    ctx.close()
