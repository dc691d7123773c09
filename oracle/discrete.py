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


# --------------------------------------------------------------------------
# the paper's own local searches: OneTwoSwap (MIS) and OneTwoFlip (MaxCut)
# --------------------------------------------------------------------------
#
# Sec. 4 describes both searches as sequential sweeps that apply a move
# whenever one exists and repeat until none does: the (1,2)-swap of Def. 2.3
# for MIS, and for MaxCut the 2-flip of Def. 2.5 alternated with the 1-flip
# of Def. 2.4.  As for the 1-flip search, the rule used on both sides is a
# parallel one: alternate (a) the 1-flip search above to a 1-flip optimum
# (for MIS: a maximal independent set, the precondition of Def. 2.3) and
# (b) one parallel iteration of the pair move, applying a set of moves whose
# gains add exactly; stop when (b) finds no move.  Every applied move raises
# the objective by at least one, so the search ends.

def _rows(graph):
    return graph.row_ptr.astype(np.int64), graph.col_idx.astype(np.int64)


def _swap_proposal(rp, ci, z, m, v):
    """Def. 2.3 move at v in I: the first pair (u, w) of v's neighbours, in
    CSR order, with m_u = m_w = 1 (v is their only neighbour in I, so
    I - v + u + w is independent iff u, w are not adjacent) and u !~ w."""
    tight = [int(u) for u in ci[rp[v]:rp[v + 1]] if z[u] == 0 and m[u] == 1]
    for i, u in enumerate(tight):
        nu = ci[rp[u]:rp[u + 1]]
        for w in tight[i + 1:]:
            k = np.searchsorted(nu, w)
            if k == len(nu) or nu[k] != w:
                return u, w
    return None


def swap_iteration_mis(graph, z, m, prio):
    """One parallel (1,2)-swap iteration on one column (z in {0,1}, m = A z
    unweighted).  Each v in I proposes its first valid pair; proposals at v
    and v' conflict when a vertex v inserts is adjacent to one v' inserts
    (the inserted sets are disjoint: an inserted vertex has one I-neighbour);
    a proposal is applied when its key (prio_v, -v) beats the key of every
    proposal it conflicts with.  Returns the list of applied (v, u, w)."""
    rp, ci = _rows(graph)
    prop, owner = {}, {}
    for v in range(graph.n):
        if z[v] == 1:
            pw = _swap_proposal(rp, ci, z, m, v)
            if pw is not None:
                prop[v] = pw
                owner[pw[0]] = v
                owner[pw[1]] = v

    def beats(a, b):
        return prio[a] > prio[b] or (prio[a] == prio[b] and a < b)

    applied = []
    for v, (u, w) in prop.items():
        lose = False
        for x in (u, w):
            for y in ci[rp[x]:rp[x + 1]]:
                o = owner.get(int(y))
                if o is not None and o != v and beats(o, v):
                    lose = True
                    break
            if lose:
                break
        if not lose:
            applied.append((v, u, w))
    return applied


def _pair_key(gain2, pv, pu, v, u):
    """Total order of 2-flip pairs: larger gain, then larger
    (prio_v + prio_u) mod 2^32, then smaller (min, max) vertex pair."""
    return (int(gain2), (int(pv) + int(pu)) & 0xFFFFFFFF, -min(v, u), -max(v, u))


def flip2_iteration_cut(graph, s, t, prio):
    """One parallel 2-flip iteration on one column (s in {-1,+1}, t = A s
    weighted).  The gain of flipping both ends of a cut edge (v, u) of
    weight w (Def. 2.5) is g_v + g_u + 2 w, g = s t the 1-flip gains: the
    edge stays cut while each single flip would uncut it.  Every v picks its
    best improving cut edge by the pair key; a pair is applied when both
    ends picked each other and no other vertex adjacent to the pair holds a
    larger best key.  Applied pairs are then non-adjacent, so their gains
    add.  Returns the list of applied (v, u)."""
    rp, ci = _rows(graph)
    w = np.ones(graph.nnz, dtype=np.int64) if graph.weight is None else graph.weight.astype(np.int64)
    g = s * t
    best = [None] * graph.n
    part = [-1] * graph.n
    for v in range(graph.n):
        for j in range(rp[v], rp[v + 1]):
            u = int(ci[j])
            if s[u] == s[v]:
                continue
            gain2 = g[v] + g[u] + 2 * w[j]
            if gain2 <= 0:
                continue
            k = _pair_key(gain2, prio[v], prio[u], v, u)
            if best[v] is None or k > best[v]:
                best[v], part[v] = k, u
    applied = []
    for v in range(graph.n):
        u = part[v]
        if u < 0 or v > u or part[u] != v:
            continue
        k = best[v]
        lose = False
        for x in (v, u):
            for y in ci[rp[x]:rp[x + 1]]:
                y = int(y)
                if y != v and y != u and best[y] is not None and best[y] > k:
                    lose = True
                    break
            if lose:
                break
        if not lose:
            applied.append((v, u))
    return applied


def flip2_iteration_cut_np(graph, s, t, prio):
    """``flip2_iteration_cut`` over whole edge arrays (numpy) for large
    graphs; same result (checked against the loop form in the tests)."""
    rp, ci = _rows(graph)
    n = graph.n
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    w = np.ones(graph.nnz, dtype=np.int64) if graph.weight is None else graph.weight.astype(np.int64)
    s = np.asarray(s, dtype=np.int64)
    g = s * np.asarray(t, dtype=np.int64)
    prio = np.asarray(prio, dtype=np.int64)
    gain2 = g[rows] + g[ci] + 2 * w
    ok = np.flatnonzero((s[rows] != s[ci]) & (gain2 > 0))
    if ok.size == 0:
        return []
    r, c = rows[ok], ci[ok]
    h = (prio[r] + prio[c]) & 0xFFFFFFFF
    mn, mx = np.minimum(r, c), np.maximum(r, c)
    # rank of every candidate edge in the pair order (both directions of a
    # pair share the key, so they share the rank)
    order = np.lexsort((-mx, -mn, h, gain2[ok]))
    key_sorted = np.stack([gain2[ok][order], h[order], -mn[order], -mx[order]], axis=1)
    new = np.ones(len(order), dtype=bool)
    new[1:] = np.any(key_sorted[1:] != key_sorted[:-1], axis=1)
    rank = np.empty(len(order), dtype=np.int64)
    rank[order] = np.cumsum(new)
    best = np.zeros(n, dtype=np.int64)  # 0 = no improving pair
    np.maximum.at(best, r, rank)
    part = np.full(n, -1, dtype=np.int64)
    top = rank == best[r]
    part[r[top]] = c[top]
    v = np.flatnonzero(part >= 0)
    u = part[v]
    cand = v[(v < u) & (part[u] == v)]
    if cand.size == 0:
        return []
    pu = part[cand]
    # largest best key among the other vertices adjacent to each end
    nb_best = np.zeros(n, dtype=np.int64)  # per vertex x: max best[y], y ~ x, y != partner(x)
    e_rows, e_cols = rows, ci
    keep = e_cols != part[e_rows]
    np.maximum.at(nb_best, e_rows[keep], best[e_cols[keep]])
    mine = best[cand]
    win = (nb_best[cand] <= mine) & (nb_best[pu] <= mine)
    return [(int(a), int(b)) for a, b in zip(cand[win], pu[win])]


def pair_search(kind, graph, Z, seed, traj, rnd, max_alternations=None):
    """OneTwoSwap (MIS) / OneTwoFlip (MaxCut) on every column, parallel rule
    above: the 1-flip search (seed, traj, rnd as for ``local_search``), then
    pair iterations with priorities of purpose SWAP for (traj, rnd, v), each
    followed by the 1-flip search again, until an iteration applies nothing.
    Returns (Z', pair moves applied per column)."""
    Z = np.array(Z, dtype=np.int64)
    n, B = Z.shape
    traj = np.asarray(traj, dtype=np.uint64)
    prio = philox.vertex_u32(seed, philox.PURPOSE_SWAP, traj[None, :], rnd,
                             np.arange(n, dtype=np.uint64)[:, None]).astype(np.int64)
    Aint = _int_adj(graph)  # MIS graphs carry no weights
    moves = np.zeros(B, dtype=np.int64)
    wsum = graph.nnz if graph.weight is None else int(np.abs(graph.weight.astype(np.int64)).sum())
    cap = max_alternations if max_alternations is not None else n + wsum + 2
    alternations = 0
    while True:
        Z = local_search(kind, graph, Z, seed, traj, rnd)[0].astype(np.int64)
        nb = Aint @ Z
        any_move = False
        for b in range(B):
            if kind == obj.MIS:
                app = swap_iteration_mis(graph, Z[:, b], nb[:, b], prio[:, b])
                for v, u, w in app:
                    Z[v, b], Z[u, b], Z[w, b] = 0, 1, 1
            else:
                it = flip2_iteration_cut if graph.n <= 4096 else flip2_iteration_cut_np
                app = it(graph, Z[:, b], nb[:, b], prio[:, b])
                for v, u in app:
                    Z[v, b], Z[u, b] = -Z[v, b], -Z[u, b]
            moves[b] += len(app)
            any_move = any_move or bool(app)
        if not any_move:
            return Z.astype(np.int8), moves
        alternations += 1
        if alternations > cap:
            raise RuntimeError("pair search did not terminate")


# --------------------------------------------------------------------------
# the pmQO pool (Alg. 3 / Alg. 4): top-K distinct solutions per graph
# --------------------------------------------------------------------------

_SM_GAMMA = 0x9E3779B97F4A7C15
_SM_M1 = 0xBF58476D1CE4E5B9
_SM_M2 = 0x94D049BB133111EB
_M64 = (1 << 64) - 1


def splitmix64(x):
    """SplitMix64 output for state x (Steele, Lea and Flood, OOPSLA 2014):
    z = x + gamma; z = (z ^ z >> 30) m1; z = (z ^ z >> 27) m2; z ^ z >> 31."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(_SM_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_SM_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_SM_M2)
        return z ^ (z >> np.uint64(31))


def solution_hash(Z):
    """Per column: sum over the vertices v in the set (z_v = 1 for MIS,
    s_v = +1 for MaxCut) of splitmix64(v), mod 2^64 (v = local index)."""
    Z = np.asarray(Z)
    h = splitmix64(np.arange(Z.shape[0], dtype=np.uint64))
    with np.errstate(over="ignore"):
        return np.where(Z > 0, h[:, None], np.uint64(0)).sum(axis=0, dtype=np.uint64)


def pool_update(kind, pool_val, pool_z, val, Z, K):
    """TopK of the pool united with the new candidates (Alg. 3 / 4): the
    union is a set, so a solution already held (equal value and hash, the
    vectors then checked equal) enters once; MIS candidates that are not
    independent (value -1) are not solutions and never enter; ranking by
    value, ties to the earlier source (pool members in rank order, then
    columns in order).  Returns (values int64[k], solutions int8[n][k])."""
    pool_val = np.asarray(pool_val, dtype=np.int64)
    cands = [(int(pool_val[i]), i, pool_z[:, i]) for i in range(len(pool_val))]
    cands += [(int(val[b]), len(pool_val) + b, Z[:, b]) for b in range(Z.shape[1])
              if not (kind == obj.MIS and val[b] < 0)]
    cands.sort(key=lambda c: (-c[0], c[1]))
    hashes = {}
    out_v, out_z = [], []
    for value, _, z in cands:
        key = (value, int(solution_hash(z.reshape(-1, 1))[0]))
        if key in hashes:
            assert np.array_equal(hashes[key], z), "hash collision between different solutions"
            continue
        hashes[key] = z
        out_v.append(value)
        out_z.append(z)
        if len(out_v) == K:
            break
    n = Z.shape[0]
    zs = np.stack(out_z, axis=1).astype(np.int8) if out_z else np.zeros((n, 0), dtype=np.int8)
    return np.array(out_v, dtype=np.int64), zs


def pool_bases(seed, traj, rnd, size):
    """Pool slot each trajectory restarts from: (u * size) >> 32 with u the
    uint32 Philox draw of purpose POOL for (traj, round)."""
    u = philox.vertex_u32(seed, philox.PURPOSE_POOL, np.asarray(traj, dtype=np.uint64), rnd, np.uint64(0))
    return ((u.astype(np.uint64) * np.uint64(size)) >> np.uint64(32)).astype(np.int64)
