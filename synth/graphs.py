"""Seeded synthetic graph generators and the canonical CSR form.

This module produces inputs only: it holds none of the method's arithmetic
(no objective, no step, no rounding, no search).  Both the oracle and the
HIP path receive the arrays it returns.

Canonical CSR (the adjacency matrix A of the notation paragraph of Sec. 2):
  * ``row_ptr``  int32[n+1], monotone, ``row_ptr[0] == 0``;
  * ``col_idx``  int32[nnz], columns sorted ascending inside every row;
  * symmetric (u in N(v) <=> v in N(u)), no self loops, no duplicates;
  * ``weight``   optional int32[nnz], symmetric (w_uv == w_vu); MaxCut only.

A batch of graphs is the block-diagonal concatenation of their CSRs with
global column indices plus ``vtx_offset`` int64[G+1].
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Graph:
    """One graph, or a block-diagonal batch of graphs, in canonical CSR."""

    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col_idx: np.ndarray  # int32[nnz]
    weight: Optional[np.ndarray] = None  # int32[nnz] or None (= unit weights)
    vtx_offset: Optional[np.ndarray] = None  # int64[G+1]; None = one graph

    def __post_init__(self):
        if self.vtx_offset is None:
            self.vtx_offset = np.array([0, self.n], dtype=np.int64)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def num_graphs(self) -> int:
        return len(self.vtx_offset) - 1

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def subgraph(self, g: int) -> "Graph":
        """Graph ``g`` of a batch, with local (0-based) column indices."""
        lo, hi = int(self.vtx_offset[g]), int(self.vtx_offset[g + 1])
        a, b = int(self.row_ptr[lo]), int(self.row_ptr[hi])
        rp = (self.row_ptr[lo:hi + 1] - a).astype(np.int32)
        ci = (self.col_idx[a:b] - lo).astype(np.int32)
        w = None if self.weight is None else self.weight[a:b].copy()
        return Graph(hi - lo, rp, ci, w)

    def edges(self):
        """Undirected edge list (u < v) with weights (1 if unweighted)."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        cols = self.col_idx.astype(np.int64)
        keep = rows < cols
        w = np.ones(self.nnz, dtype=np.int64) if self.weight is None else self.weight.astype(np.int64)
        return rows[keep], cols[keep], w[keep]


def from_edges(n: int, u, v, w=None) -> Graph:
    """Canonical CSR from an undirected edge list.

    Self loops are dropped; duplicate pairs keep their first weight.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if w is None:
        w = np.ones(len(u), dtype=np.int64)
        weighted = False
    else:
        w = np.asarray(w, dtype=np.int64)
        weighted = True
    keep = u != v
    u, v, w = u[keep], v[keep], w[keep]
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    key = a * n + b
    _, first = np.unique(key, return_index=True)
    a, b, w = a[first], b[first], w[first]
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    ws = np.concatenate([w, w])
    order = np.lexsort((cols, rows))
    rows, cols, ws = rows[order], cols[order], ws[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32")
    return Graph(n, row_ptr.astype(np.int32), cols.astype(np.int32),
                 ws.astype(np.int32) if weighted else None)


def concat(graphs: Sequence[Graph]) -> Graph:
    """Block-diagonal batch of graphs (global column indices)."""
    offs = np.zeros(len(graphs) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([g.n for g in graphs])
    nnz_offs = np.zeros(len(graphs) + 1, dtype=np.int64)
    nnz_offs[1:] = np.cumsum([g.nnz for g in graphs])
    if nnz_offs[-1] >= 2**31:
        raise ValueError("total nnz does not fit int32")
    rp = np.concatenate([np.asarray(g.row_ptr[:-1], dtype=np.int64) + nnz_offs[i]
                         for i, g in enumerate(graphs)] + [nnz_offs[-1:]])
    ci = np.concatenate([np.asarray(g.col_idx, dtype=np.int64) + offs[i]
                         for i, g in enumerate(graphs)])
    weighted = [g.weight is not None for g in graphs]
    if any(weighted) and not all(weighted):
        raise ValueError("mixed weighted and unweighted graphs")
    w = np.concatenate([g.weight for g in graphs]).astype(np.int32) if all(weighted) else None
    return Graph(int(offs[-1]), rp.astype(np.int32), ci.astype(np.int32), w, offs)


# --------------------------------------------------------------------------
# generators
# --------------------------------------------------------------------------

def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def erdos_renyi(n: int, p: float, seed: int) -> Graph:
    """G(n, p): every unordered pair is an edge independently with prob. p.

    Small n enumerates all pairs; large n skips between successes with
    geometric gaps over the lower-triangle pair index (Batagelj & Brandes,
    Phys. Rev. E 71, 2005), which has the same distribution.
    """
    rng = _rng(seed)
    npairs = n * (n - 1) // 2
    if n <= 4096:
        iu, ju = np.triu_indices(n, k=1)
        keep = rng.random(len(iu)) < p
        return from_edges(n, iu[keep], ju[keep])
    if p <= 0.0:
        return from_edges(n, [], [])
    chunks = []
    pos = -1
    expected = int(npairs * p)
    while True:
        m = max(1024, int(1.1 * (expected - sum(len(c) for c in chunks))) + 1024)
        gaps = rng.geometric(p, size=m).astype(np.int64)
        idx = pos + np.cumsum(gaps)
        if idx[-1] >= npairs:
            chunks.append(idx[idx < npairs])
            break
        chunks.append(idx)
        pos = int(idx[-1])
    lin = np.concatenate(chunks)
    # pair index L -> (a, b) with b < a, L = a*(a-1)/2 + b
    a = np.floor((1.0 + np.sqrt(1.0 + 8.0 * lin.astype(np.float64))) / 2.0).astype(np.int64)
    a = np.where(a * (a - 1) // 2 > lin, a - 1, a)
    a = np.where((a + 1) * a // 2 <= lin, a + 1, a)
    b = lin - a * (a - 1) // 2
    return from_edges(n, a, b)


def random_regular(n: int, d: int, seed: int) -> Graph:
    """Random d-regular simple graph by the pairing (configuration) model.

    Stubs are paired uniformly; stubs that end in a self loop or a repeated
    pair are re-paired together with an equal number of randomly chosen
    good pairs until the pairing is simple.
    """
    if (n * d) % 2:
        raise ValueError("n*d must be even")
    rng = _rng(seed)
    stubs = np.repeat(np.arange(n, dtype=np.int64), d)
    rng.shuffle(stubs)
    a, b = stubs[0::2].copy(), stubs[1::2].copy()
    for _ in range(10000):
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        key = lo * n + hi
        order = np.argsort(key, kind="stable")
        sk = key[order]
        dup = np.zeros(len(a), dtype=bool)
        dup[order[1:]] = sk[1:] == sk[:-1]
        bad = (a == b) | dup
        nb = int(bad.sum())
        if nb == 0:
            return from_edges(n, a, b)
        good_idx = np.flatnonzero(~bad)
        extra = rng.choice(good_idx, size=min(len(good_idx), max(nb, 4)), replace=False)
        sel = np.concatenate([np.flatnonzero(bad), extra])
        pool = np.concatenate([a[sel], b[sel]])
        rng.shuffle(pool)
        a[sel], b[sel] = pool[0::2], pool[1::2]
    raise RuntimeError("pairing model did not converge")


def barabasi_albert(n: int, m: int, seed: int) -> Graph:
    """Preferential attachment: a seed clique K_{m+1}, then every new vertex
    joins m distinct existing vertices drawn with probability proportional
    to their degree (Barabasi & Albert, Science 1999)."""
    rng = _rng(seed)
    src, dst = [], []
    targets = []  # vertex list with multiplicity = degree
    for i in range(m + 1):
        for j in range(i + 1, m + 1):
            src.append(i)
            dst.append(j)
            targets += [i, j]
    tgt = np.empty(2 * m * n + len(targets), dtype=np.int64)
    tgt[:len(targets)] = targets
    tlen = len(targets)
    src_arr = np.empty(m * (n - m - 1), dtype=np.int64)
    dst_arr = np.empty(m * (n - m - 1), dtype=np.int64)
    e = 0
    for v in range(m + 1, n):
        chosen = set()
        while len(chosen) < m:
            draw = tgt[rng.integers(0, tlen, size=2 * m)]
            for u in draw:
                if len(chosen) < m:
                    chosen.add(int(u))
        for u in sorted(chosen):
            src_arr[e] = v
            dst_arr[e] = u
            e += 1
            tgt[tlen] = v
            tgt[tlen + 1] = u
            tlen += 2
    u = np.concatenate([np.asarray(src, dtype=np.int64), src_arr[:e]])
    w = np.concatenate([np.asarray(dst, dtype=np.int64), dst_arr[:e]])
    return from_edges(n, u, w)


def torus_pm1(side: int, seed: int) -> Graph:
    """side x side 2-D torus (right and down neighbours, wrap-around) with
    edge weights +1 or -1, each with probability 1/2."""
    rng = _rng(seed)
    n = side * side
    r, c = np.divmod(np.arange(n, dtype=np.int64), side)
    right = r * side + (c + 1) % side
    down = ((r + 1) % side) * side + c
    u = np.concatenate([np.arange(n), np.arange(n)])
    v = np.concatenate([right, down])
    w = np.where(rng.random(2 * n) < 0.5, 1, -1)
    return from_edges(n, u, v, w)


def er_batch(count: int, n_lo: int, n_hi: int, p: float, seed: int) -> Graph:
    """``count`` independent G(n_g, p) graphs, n_g uniform in [n_lo, n_hi],
    as one block-diagonal batch (graph i uses seed ``seed + i``)."""
    rng = _rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, size=count)
    return concat([erdos_renyi(int(s), p, seed + 1 + i) for i, s in enumerate(sizes)])


# small named graphs used by tests
def path(n: int) -> Graph:
    return from_edges(n, np.arange(n - 1), np.arange(1, n))


def cycle(n: int) -> Graph:
    return from_edges(n, np.arange(n), (np.arange(n) + 1) % n)


def complete(n: int) -> Graph:
    iu, ju = np.triu_indices(n, k=1)
    return from_edges(n, iu, ju)


def star(leaves: int) -> Graph:
    return from_edges(leaves + 1, np.zeros(leaves, dtype=np.int64), np.arange(1, leaves + 1))


def empty(n: int) -> Graph:
    return from_edges(n, [], [])


def with_weights(g: Graph, seed: int, values=(-1, 1)) -> Graph:
    """Same graph with symmetric weights drawn uniformly from ``values``."""
    rng = _rng(seed)
    ru, rv, _ = g.edges()
    w = rng.choice(np.asarray(values, dtype=np.int64), size=len(ru))
    return from_edges(g.n, ru, rv, w)
