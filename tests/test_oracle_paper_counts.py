"""The oracle against the operation counts the paper prints for its softened
1024-body Plummer sphere (Sec. 3.1): the first global time step of the CC
method evaluates about 6.6e8 pair time steps, 1.1e9 kicks and 5.0e6 drifts
(tests/golden/paper_plummer1024_first_step.txt).

Our initial conditions are another realisation of the same model (the
paper's are not published), so the counts agree statistically: across
seeds they scatter by a few per cent.  Reading of "kick evaluations": one
per particle and partner, i.e. two per kicked pair (the pair force acts on
both members).  A mistake in the time-step criterion (eta in the wrong
place, a dropped symmetrisation term, a non-strict threshold) or in the
recursion changes these counts by factors, not per cent."""
import pytest

import oracle
import synth

from .golden import load_golden


@pytest.fixture(scope="module")
def paper():
    (rec,) = load_golden("paper_plummer1024_first_step.txt")
    return rec


@pytest.fixture(scope="module")
def first_step(paper):
    s = synth.plummer(int(paper["n"]), 1)
    p = oracle.Params(eta=paper["eta"], eps2=paper["eps"] ** 2)
    rc, st = oracle.evolve(s, paper["dt"], paper["dt"], p)
    return st


def test_cc_first_step_counts_match_the_paper(paper, first_step):
    st = first_step
    assert abs(st["tau_evals"] / paper["tau_evals"] - 1) < 0.10, st["tau_evals"]
    assert abs(st["drifts"] / paper["drifts"] - 1) < 0.10, st["drifts"]
    assert abs(2 * st["kick_pairs"] / paper["kicks"] - 1) < 0.15, st["kick_pairs"]
