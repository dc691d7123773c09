"""Exhaustive answers on tiny graphs (n <= 20), straight from the problem
definitions (Def. 2.1 MIS, Def. 2.2 MaxCut).  Test infrastructure only."""
from __future__ import annotations

import itertools

import numpy as np


def all_binary(n):
    """All 2^n vectors in {0,1}^n as rows (int8)."""
    return np.array(list(itertools.product((0, 1), repeat=n)), dtype=np.int8)


def _edges(graph):
    u, v, w = graph.edges()
    return u, v, w


def independence_number(graph):
    """alpha(G): the largest |I| over all independent sets."""
    Z = all_binary(graph.n)
    u, v, _ = _edges(graph)
    indep = ~np.any((Z[:, u] == 1) & (Z[:, v] == 1), axis=1)
    return int(Z[indep].sum(axis=1).max())


def maximal_independent_sets(graph):
    """Set of maximal independent sets, each as a tuple of 0/1."""
    Z = all_binary(graph.n).astype(np.int64)
    u, v, _ = _edges(graph)
    out = set()
    for z in Z:
        if np.any((z[u] == 1) & (z[v] == 1)):
            continue
        covered = z.copy()
        covered[u[z[v] == 1]] = 1
        covered[v[z[u] == 1]] = 1
        if np.all(covered == 1):
            out.add(tuple(int(x) for x in z))
    return out


def max_cut(graph):
    """max over S of the total weight of the edges crossing (S, V \\ S)."""
    Z = all_binary(graph.n)
    u, v, w = _edges(graph)
    cuts = ((Z[:, u] != Z[:, v]) * w[None, :]).sum(axis=1)
    return int(cuts.max())
