"""The paper's trends on the GPU (trend-only: its figures carry no printed
values): the softened Plummer sphere's energy error is second order in eta
under both splits, with HOLD evaluating more pair steps than CC (Sec. 3.1);
in box fractals the CC split's pair-step count stays flat as the fractal
dimension falls while HOLD's grows (Sec. 3.3)."""
import math

import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1407_7105_amd import Context, State  # noqa: E402


def run(p, dt0, t_end, **kw):
    ctx = Context(device=0, **kw)
    s = State.from_numpy(p)
    e0 = ctx.diagnostics(s)["energy"]
    st = ctx.evolve(s, dt0, t_end)
    e1 = ctx.diagnostics(s)["energy"]
    ctx.close()
    return abs(e1 / e0 - 1), st


def test_softened_plummer_second_order_and_hold_costlier():
    p = synth.plummer(1024, 1)
    etas = (0.01, 0.03, 0.1)
    for hold in (0, 1):
        errs = []
        for eta in etas:
            de, st = run(p, 1 / 64, 1.0, eta=eta, eps2=(1 / 256) ** 2, hold=hold)
            errs.append(de)
        slopes = [math.log(errs[k + 1] / errs[k]) / math.log(etas[k + 1] / etas[k]) for k in range(2)]
        assert all(1.5 < s < 2.6 for s in slopes), (hold, errs, slopes)
    _, cc = run(p, 1 / 64, 0.25, eta=0.01, eps2=(1 / 256) ** 2)
    _, ho = run(p, 1 / 64, 0.25, eta=0.01, eps2=(1 / 256) ** 2, hold=1)
    # HOLD needs every pair of every split; the CC count here is the sweep's
    # n(n-1)/2 per non-star split (the paper's BFS needs fewer still)
    assert ho["tau_pairs_alg"] > 1.2 * cc["tau_pairs_alg"]


def test_fractal_dimension_trend_of_pair_steps():
    taus = {}
    for dim in (1.6, 3.0):
        p = synth.fractal(1024, 100 * int(10 * dim) + 1, dim=dim)
        for name, kw in (("cc", {}), ("hold", {"hold": 1})):
            _, st = run(p, 1 / 64, 0.25, eta=0.03, **kw)
            taus[(dim, name)] = st["tau_pairs_alg"]
    # CC: flat (here falling) as the dimension drops; HOLD: several times more
    assert taus[(1.6, "cc")] < 1.5 * taus[(3.0, "cc")], taus
    assert taus[(1.6, "hold")] > 3.0 * taus[(3.0, "hold")], taus
    assert taus[(1.6, "hold")] > 4.0 * taus[(1.6, "cc")], taus
