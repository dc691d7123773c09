"""Exact integer side of the method: rounding, evaluation, the MIS checker,
1-flip gains, local search and the mutation reset.

Arrays are vertex-major [n][B]: column b is one trajectory.  MIS solutions
are z in {0,1}; MaxCut solutions are s in {-1,+1}.
Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import objectives as obj
from . import philox


def _int_adj(graph):
    data = np.ones(graph.nnz, dtype=np.int64) if graph.weight is None else graph.weight.astype(np.int64)
    return sp.csr_matrix((data, graph.col_idx.astype(np.int64), graph.row_ptr.astype(np.int64)),
                         shape=(graph.n, graph.n))


# --------------------------------------------------------------------------
# rounding (Sec. 3: I = {x_v > 0.5} on [0,1]^n, S = {x_v > 0} on [-1,1]^n)
# --------------------------------------------------------------------------

def round_mis(X):
    return (np.asarray(X) > 0.5).astype(np.int8)


def round_cut(X):
    return np.where(np.asarray(X) > 0, 1, -1).astype(np.int8)


def round_x(kind, X):
    return round_mis(X) if kind == obj.MIS else round_cut(X)


# --------------------------------------------------------------------------
# evaluation
# --------------------------------------------------------------------------

def neighbour_counts(graph, Z):
    """m_v = |N(v) cap I| (MIS, proof of Prop. 3.1) or t_v = (A s)_v (MaxCut,
    proof of Prop. 3.4), exact int64."""
    return _int_adj(graph) @ np.asarray(Z, dtype=np.int64)


def evaluate_mis(graph, Z):
    """(|I|, number of edges inside I) per column (Def. 2.1, Eq. (1))."""
    Z = np.asarray(Z, dtype=np.int64)
    m = neighbour_counts(graph, Z)
    return Z.sum(axis=0), (Z * m).sum(axis=0) // 2


def evaluate_cut(graph, S):
    """Cut(S) per column: total weight of the edges whose ends differ (Def. 2.2)."""
    S = np.asarray(S, dtype=np.int64)
    u, v, w = graph.edges()
    return ((S[u] != S[v]) * w[:, None]).sum(axis=0)


def value(kind, graph, Z):
    """The discrete objective the search accepts on (Sec. 4): the MIS size
    when the set is independent (else -1), the cut value for MaxCut."""
    if kind == obj.MIS:
        size, conf = evaluate_mis(graph, Z)
        return np.where(conf == 0, size, -1).astype(np.int64)
    return evaluate_cut(graph, Z).astype(np.int64)


def is_pga_fixed_mis(graph, Z, gamma, alpha=1.0):
    """The checker of Eq. (8): 1{x = Pi_[0,1](x + alpha grad h(x))} on a binary x,
    evaluated literally in float64, per column."""
    A = obj.adjacency(graph)
    X = np.asarray(Z, dtype=np.float64)
    Y = np.clip(X + alpha * obj.grad_h(X, A, gamma), 0.0, 1.0)
    return np.all(Y == X, axis=0)


def is_pga_fixed_cut(graph, S, lam, alpha=1.0):
    """A binary s in {-1,+1}^n is a fixed point of the projected step on
    f_B (Eq. (7), Sec. 3): 1{s = Pi_[-1,1](s + alpha grad f_B(s))}, evaluated
    literally in float64, per column."""
    A = obj.adjacency(graph)
    X = np.asarray(S, dtype=np.float64)
    Y = np.clip(X + alpha * obj.grad_f_B(X, A, lam), -1.0, 1.0)
    return np.all(Y == X, axis=0)


def is_pga_fixed(kind, graph, Z, param, alpha=1.0):
    """The early-exit test of the schedule: the rounded point is a fixed point
    of the projected gradient step (Eq. (8) for MIS, its f_B analogue for
    MaxCut)."""
    if kind == obj.MIS:
        return is_pga_fixed_mis(graph, Z, param, alpha)
    return is_pga_fixed_cut(graph, Z, param, alpha)


def is_maximal_independent(graph, Z):
    """Brute definition: no edge inside I, and every v outside I has a
    neighbour in I."""
    Z = np.asarray(Z, dtype=np.int64)
    m = neighbour_counts(graph, Z)
    return np.all(np.where(Z == 1, m == 0, m >= 1), axis=0)


# --------------------------------------------------------------------------
# 1-flip gains
# --------------------------------------------------------------------------

def gains(kind, graph, Z, gamma=2.0):
    """Exact objective change of flipping vertex v alone.

    MaxCut: Cut(s with s_v negated) - Cut(s) = s_v (A s)_v (the 1-flip gain
    identity in the proof of Prop. 3.4, divided by 4 since the cut is
    (1/4) x^T L x and f_A differs from it by a constant).
    MIS (penalised h of Eq. (3) at binary z): adding v not in I gives
    1 - gamma m_v, removing v in I gives gamma m_v - 1."""
    nb = neighbour_counts(graph, Z)
    Z = np.asarray(Z, dtype=np.int64)
    if kind == obj.MIS:
        return np.where(Z == 1, gamma * nb - 1.0, 1.0 - gamma * nb)
    return Z * nb


# --------------------------------------------------------------------------
# local search
# --------------------------------------------------------------------------

def _ls_keys(kind, Z, nb):
    """Positive-gain set P and the integer first key component."""
    if kind == obj.MIS:
        P = ((Z == 1) & (nb >= 1)) | ((Z == 0) & (nb == 0))
        k1 = np.where(Z == 1, nb, 0)
    else:
        k1 = Z * nb
        P = k1 > 0
    return P, k1


def local_search(kind, graph, Z, seed, traj, rnd, max_iters=None, stop_after=None):
    """1-flip local search with per-vertex gain vectors, parallel rule.

    The paper's search visits vertices one after another and repeats until
    no move applies (Sec. 4, description of OneTwoSwap / OneTwoFlip).  A
    sequential visit order cannot be reproduced by a parallel machine, so
    the rule used on both sides is: in every iteration
      P = vertices whose flip has positive gain
          (MIS: v in I with m_v >= 1, or v not in I with m_v = 0;
           MaxCut: s_v t_v > 0),
      F = v in P whose key beats the key of every neighbour in P, with the
          key ordered lexicographically as (k1, prio, -v), k1 = m_v for a
          removal, 0 for an addition (MIS) or the gain (MaxCut), and prio
          the uint32 Philox draw of purpose LS for (traj, round, v);
    all of F flips at once (F is independent, so the gains add) and the
    neighbour counts are updated; stop when P is empty (or after
    ``stop_after`` iterations, for tests).
    Returns (Z', iterations)."""
    Z = np.array(Z, dtype=np.int64)
    n, B = Z.shape
    Aint = _int_adj(graph)
    nb = Aint @ Z
    prio = philox.vertex_u32(seed, philox.PURPOSE_LS, np.asarray(traj, dtype=np.uint64)[None, :], rnd,
                             np.arange(n, dtype=np.uint64)[:, None]).astype(np.int64)
    rows = np.repeat(np.arange(n), np.diff(graph.row_ptr))
    cols = graph.col_idx.astype(np.int64)
    it = 0
    limit = max_iters if max_iters is not None else 4 * (n + graph.nnz) + 64
    while True:
        P, k1 = _ls_keys(kind, Z, nb)
        if not P.any() or (stop_after is not None and it >= stop_after):
            return Z.astype(np.int8), it
        if it >= limit:
            raise RuntimeError("local search did not terminate")
        # does neighbour u (= cols) beat v (= rows)?  lexicographic (k1, prio, -v)
        ku, kv = k1[cols], k1[rows]
        pu, pv = prio[cols], prio[rows]
        beats = (ku > kv) | ((ku == kv) & ((pu > pv) | ((pu == pv) & (cols[:, None] < rows[:, None]))))
        beaten = np.zeros_like(P)
        np.logical_or.at(beaten, rows, P[cols] & beats)
        F = P & ~beaten
        old = Z.copy()
        if kind == obj.MIS:
            Z = np.where(F, 1 - Z, Z)
        else:
            Z = np.where(F, -Z, Z)
        nb = nb + Aint @ (Z - old)
        it += 1


def local_search_sequential(kind, graph, z, gamma=2.0):
    """The paper's sequential form for one column: sweep v = 0..n-1, flip v
    whenever its gain is positive, repeat sweeps until a full sweep makes
    no move.  Used to check that both forms end at 1-flip local optima."""
    z = np.array(z, dtype=np.int64)
    A = _int_adj(graph)
    nb = A @ z
    rp, ci = graph.row_ptr, graph.col_idx
    w = np.ones(graph.nnz, dtype=np.int64) if graph.weight is None else graph.weight.astype(np.int64)
    moved = True
    while moved:
        moved = False
        for v in range(graph.n):
            if kind == obj.MIS:
                gain = gamma * nb[v] - 1 if z[v] == 1 else 1 - gamma * nb[v]
            else:
                gain = z[v] * nb[v]
            if gain > 0:
                old = z[v]
                z[v] = 1 - z[v] if kind == obj.MIS else -z[v]
                d = z[v] - old
                for j in range(rp[v], rp[v + 1]):
                    nb[ci[j]] += w[j] * d
                moved = True
    return z.astype(np.int8)


# --------------------------------------------------------------------------
# mutation reset (Sec. 4)
# --------------------------------------------------------------------------

def reset_count(rho, n):
    """|R| = floor(rho n), rho a float64."""
    return int(np.floor(float(rho) * n))


def reset_set(n, k, seed, traj, rnd, keys=None):
    """R for every column: the k vertices with the smallest (key, v), key
    the uint32 Philox draw of purpose RESET for (traj, round, v) (or the
    given ``keys`` [n][B]).  The k smallest of i.i.d. keys form a uniformly
    random k-subset; equal keys fall to the lower index.  Returns bool [n][B]."""
    traj = np.asarray(traj, dtype=np.uint64)
    if keys is None:
        keys = philox.vertex_u32(seed, philox.PURPOSE_RESET, traj[None, :], rnd,
                                 np.arange(n, dtype=np.uint64)[:, None])
    keys = np.asarray(keys)
    B = keys.shape[1]
    mask = np.zeros((n, B), dtype=bool)
    v = np.arange(n)
    for b in range(B):
        order = np.lexsort((v, keys[:, b]))
        mask[order[:k], b] = True
    return mask


def reset_apply(kind, Zbest, mask, mode="zero"):
    """x from the incumbent (Alg. 1 / Alg. 2: x_v = 1(v in I_sol) or +-1),
    then x_R <- 0 (the paper's reset, Sec. 4), or in ``flip`` mode x_R is
    the complement (1 - z or -s)."""
    base = np.asarray(Zbest, dtype=np.float32)
    if mode == "zero":
        rv = np.zeros_like(base)
    elif kind == obj.MIS:
        rv = np.float32(1.0) - base
    else:
        rv = -base
    return np.where(mask, rv, base).astype(np.float32)
