"""Neural bounding hierarchies (test infrastructure; see oracle/__init__).

Sec. 3.3: bounds can be stacked into a tree like a bounding volume
hierarchy; the tree is given by the user and every node's network bounds,
conservatively, what lies below it, so a query can stop descending wherever
a node says "no".  The reading used here (the paper gives no formula):

  * node v's bound is meant to contain the union of the indicators of the
    leaves below v (a leaf bounds its own object);
  * a region r is reported for leaf l iff h_v(r) = 1 for every node v on the
    path from the root to l, both ends included; the decision of a node is
    the single bound's, h = !(z < tau).

Trees are described breadth first with node 0 the root: node p's children
are child_begin[p] .. child_end[p]-1, and these ranges, taken in the order
of p, are exactly 1 .. n-1.  Leaves (empty ranges) are ranked in node order.
"""

from __future__ import annotations

import numpy as np


def structure(child_begin, child_end):
    """(parent, level, leaves): parent[0] = -1, level of every node, and the
    leaf nodes in rank order.  Raises ValueError for a malformed tree."""
    cb = [int(x) for x in child_begin]
    ce = [int(x) for x in child_end]
    n = len(cb)
    if n == 0 or len(ce) != n:
        raise ValueError("need one child range per node")
    parent = [-1] * n
    level = [0] * n
    nxt = 1
    for p in range(n):
        if ce[p] < cb[p]:
            raise ValueError(f"node {p}: reversed child range")
        if ce[p] == cb[p]:
            continue
        if cb[p] != nxt or ce[p] > n or cb[p] <= p:
            raise ValueError(f"node {p}: children are not the next nodes in breadth-first order")
        for c in range(cb[p], ce[p]):
            parent[c] = p
            level[c] = level[p] + 1
        nxt = ce[p]
    if nxt != n:
        raise ValueError("some nodes have no parent")
    leaves = [p for p in range(n) if cb[p] == ce[p]]
    return parent, level, leaves


def traverse(decide, child_begin, child_end, n_rows: int):
    """Descend from the root: decide(node, rows) gives the node's decisions
    (bool array) for the row indices `rows`; returns, per leaf rank, the
    sorted rows that every node on the leaf's path accepts."""
    _, _, leaves = structure(child_begin, child_end)
    rank = {v: i for i, v in enumerate(leaves)}
    out = [np.zeros(0, dtype=np.int64) for _ in leaves]

    def visit(v, rows):
        if rows.size == 0:
            return
        keep = rows[np.asarray(decide(v, rows), dtype=bool)]
        if child_begin[v] == child_end[v]:
            out[rank[v]] = keep
            return
        for c in range(int(child_begin[v]), int(child_end[v])):
            visit(c, keep)

    visit(0, np.arange(n_rows, dtype=np.int64))
    return out
