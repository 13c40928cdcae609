"""Pins of the hierarchy oracle (Sec. 3.3): the level-by-level descent is
checked against the definition written differently -- for every leaf, the
AND of all decisions on its root path, found by walking parent links up --
on random trees and random decision tables, plus hand-built trees and the
all-accept / all-reject cases."""

import numpy as np
import pytest

from oracle import hierarchy as H


def random_tree(rng, n_max=40, fan_max=5):
    """A random breadth-first tree: each node in turn gets 0..fan_max
    children while nodes remain."""
    n = int(rng.integers(1, n_max + 1))
    cb, ce = [0] * n, [0] * n
    nxt = 1
    for p in range(n):
        k = int(rng.integers(0, fan_max + 1)) if nxt < n else 0
        if p == nxt - 1 and nxt < n and k == 0:
            k = 1        # keep the tree connected: the last node so far must have a child
        k = min(k, n - nxt)
        cb[p], ce[p] = (nxt, nxt + k) if k else (0, 0)
        nxt += k
    return cb, ce


def path_and(D, parent, leaf):
    ok = D[leaf].copy()
    v = parent[leaf]
    while v >= 0:
        ok &= D[v]
        v = parent[v]
    return np.nonzero(ok)[0]


def test_structure_of_a_hand_built_tree():
    #        0
    #     /  |  \
    #    1   2   3
    #   / \     /|\
    #  4   5   6 7 8
    #          |
    #          9
    cb = [1, 4, 0, 6, 0, 0, 9, 0, 0, 0]
    ce = [4, 6, 0, 9, 0, 0, 10, 0, 0, 0]
    parent, level, leaves = H.structure(cb, ce)
    assert parent == [-1, 0, 0, 0, 1, 1, 3, 3, 3, 6]
    assert level == [0, 1, 1, 1, 2, 2, 2, 2, 2, 3]
    assert leaves == [2, 4, 5, 7, 8, 9]


@pytest.mark.parametrize("cb,ce", [
    ([2, 0, 0], [3, 0, 0]),          # node 1 has no parent
    ([1, 0], [3, 0]),                # range beyond the last node
    ([1, 2, 0, 0], [2, 4, 0, 0]),    # fine ...
])
def test_structure_rejects_malformed_trees(cb, ce):
    if cb == [1, 2, 0, 0]:
        assert H.structure(cb, ce)[2] == [2, 3]
        return
    with pytest.raises(ValueError):
        H.structure(cb, ce)


def test_structure_rejects_out_of_order_children():
    # node 0's children are 1, 2; node 2's children listed before node 1's
    with pytest.raises(ValueError):
        H.structure([1, 5, 3, 0, 0, 0], [3, 6, 5, 0, 0, 0])


@pytest.mark.parametrize("seed", range(12))
def test_descent_equals_the_and_over_root_paths(seed):
    rng = np.random.default_rng(seed)
    cb, ce = random_tree(rng)
    parent, _, leaves = H.structure(cb, ce)
    n_rows = int(rng.integers(1, 300))
    D = rng.random((len(cb), n_rows)) < rng.uniform(0.3, 0.95)
    calls = []

    def decide(v, rows):
        calls.append((v, rows.size))
        return D[v, rows]

    out = H.traverse(decide, cb, ce, n_rows)
    assert len(out) == len(leaves)
    for r, leaf in enumerate(leaves):
        assert np.array_equal(out[r], path_and(D, parent, leaf)), (seed, leaf)
        assert np.all(np.diff(out[r]) > 0)
    # a node is only asked about the rows all of its ancestors accepted
    for v, m in calls:
        if parent[v] >= 0:
            assert m <= n_rows


def test_accept_all_and_reject_subtree():
    cb = [1, 3, 0, 0, 0]
    ce = [3, 5, 0, 0, 0]
    _, _, leaves = H.structure(cb, ce)
    assert leaves == [2, 3, 4]
    out = H.traverse(lambda v, rows: np.ones(rows.size, bool), cb, ce, 7)
    assert all(np.array_equal(o, np.arange(7)) for o in out)
    # node 1 rejects everything: its leaves 3 and 4 get nothing, leaf 2 all
    out = H.traverse(lambda v, rows: np.full(rows.size, v != 1), cb, ce, 7)
    assert np.array_equal(out[0], np.arange(7)) and out[1].size == 0 and out[2].size == 0


def test_single_node_tree_is_the_plain_decision():
    d = np.array([1, 0, 0, 1, 1, 0, 1], bool)
    out = H.traverse(lambda v, rows: d[rows], [0], [0], d.size)
    assert np.array_equal(out[0], np.nonzero(d)[0])
