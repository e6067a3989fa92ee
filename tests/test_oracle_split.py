"""Pins of the oracle's connected-component split (eq. 20, Sec. 2.3):
breadth-first search, union-find and a transitive closure must agree, the
fully connected case costs n-1 evaluations, and labels are canonical."""
import numpy as np
import pytest

import oracle
from synth import Particles, plummer


def random_set(n, seed, spread=1.0):
    rng = np.random.default_rng(seed)
    pos = rng.normal(size=(n, 3)) * spread * rng.uniform(0.05, 1.0, (n, 1))
    vel = rng.normal(size=(n, 3))
    return Particles.from_arrays(pos, vel, rng.uniform(0.2, 1.0, n) / n)


def tau_matrix(s, p):
    n = len(s.m)
    pi, pj = np.triu_indices(n, 1)
    t = oracle.pair_timesteps(s, pi.astype(np.int32), pj.astype(np.int32), p)
    T = np.full((n, n), np.inf)
    T[pi, pj] = t
    T[pj, pi] = t
    return T


def closure_labels(adj):
    """Floyd-Warshall transitive closure; label = smallest reachable index."""
    n = adj.shape[0]
    R = adj.copy() | np.eye(n, dtype=bool)
    for k in range(n):
        R |= R[:, k:k + 1] & R[k:k + 1, :]
    return np.array([int(np.flatnonzero(R[i])[0]) for i in range(n)])


@pytest.mark.parametrize("seed", range(12))
def test_bfs_uf_closure_agree(seed):
    n = 4 + seed % 13
    s = random_set(n, seed)
    p = oracle.Params(eta=0.01)
    T = tau_matrix(s, p)
    finite = np.sort(T[np.isfinite(T)])
    for q in (0.1, 0.3, 0.5, 0.7, 0.9):
        h = float(finite[int(q * (len(finite) - 1))])
        want = closure_labels(T < h)
        bfs, _ = oracle.split_bfs(s, h, p=p)
        uf = oracle.split_uf(s, h, p=p)
        np.testing.assert_array_equal(bfs, want)
        np.testing.assert_array_equal(uf, want)


def test_edge_is_strict_at_threshold():
    # h equal to a pair's tau is not an edge; the next double above is (eq. 20)
    s = random_set(2, 1)
    p = oracle.Params(eta=0.01)
    t = oracle.tau(s, 0, 1, p)
    lab, _ = oracle.split_bfs(s, t, p=p)
    assert list(lab) == [0, 1]
    lab, _ = oracle.split_bfs(s, float(np.nextafter(t, np.inf)), p=p)
    assert list(lab) == [0, 0]


def test_fully_connected_costs_n_minus_1():
    # Sec. 2.3: if every pair is below h one pass from any X assigns all particles
    s = random_set(40, 7)
    p = oracle.Params(eta=0.01)
    T = tau_matrix(s, p)
    h = float(np.max(T[np.isfinite(T)])) * 2.0
    lab, ev = oracle.split_bfs(s, h, p=p)
    assert np.all(lab == 0) and ev == 39


def test_all_slow_gives_singletons():
    s = random_set(30, 8)
    p = oracle.Params(eta=0.01)
    T = tau_matrix(s, p)
    h = float(np.min(T)) * 0.5
    lab, ev = oracle.split_bfs(s, h, p=p)
    np.testing.assert_array_equal(lab, np.arange(30))
    assert ev == 30 * 29 // 2


def test_permutation_invariance():
    s = random_set(60, 9)
    p = oracle.Params(eta=0.01)
    T = tau_matrix(s, p)
    h = float(np.median(T[np.isfinite(T)])) * 0.05
    lab, _ = oracle.split_bfs(s, h, p=p)
    perm = np.random.default_rng(1).permutation(60)
    sp = Particles(*(a[perm].copy() for a in s.arrays()))
    labp, _ = oracle.split_bfs(sp, h, p=p)
    # same partition: particles perm[a], perm[b] together iff a, b together
    A = lab[:, None] == lab[None, :]
    B = labp[:, None] == labp[None, :]
    inv = np.argsort(perm)
    np.testing.assert_array_equal(A, B[np.ix_(inv, inv)])


def test_subset_labels_use_original_indices():
    s = random_set(20, 10)
    p = oracle.Params(eta=0.01)
    I = np.array([3, 5, 6, 11, 17], np.int64)
    T = tau_matrix(s, p)[np.ix_(I, I)]
    h = float(np.median(T[np.isfinite(T)]))
    lab, _ = oracle.split_bfs(s, h, I=I, p=p)
    want = I[closure_labels(T < h)]
    np.testing.assert_array_equal(lab, want)


def test_split_labels_all_particles():
    s = plummer(128, 5)
    p = oracle.Params(eta=0.01)
    lab, nt, ev = oracle.split_labels(s, 1.0 / 256, p)
    cnt = np.bincount(lab, minlength=128)
    assert nt == int(np.sum(cnt >= 2))
    uf = oracle.split_uf(s, 1.0 / 256, p=p)
    np.testing.assert_array_equal(lab, uf)
    assert np.all(lab <= np.arange(128))
