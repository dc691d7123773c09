"""Pins of the oracle's OneTwoSwap / OneTwoFlip (Def. 2.3, Def. 2.5, the
search description of Sec. 4).  The checks recompute independence, set
sizes and cut values from the definitions by brute force over every move,
so they do not reuse the gain formulas the searches use.  CPU only."""
import itertools

import numpy as np
import pytest

from synth import graphs
from oracle import discrete


def _adj_sets(g):
    rp, ci = g.row_ptr, g.col_idx
    return [set(int(u) for u in ci[rp[v]:rp[v + 1]]) for v in range(g.n)]


def _independent(nbr, I):
    return all(not (nbr[v] & I) for v in I)


def _swap_repairable(g, z):
    """Def. 2.3 by brute force: some v in I and two neighbours u, w not in I
    such that I - v + u + w is independent."""
    nbr = _adj_sets(g)
    I = set(int(v) for v in np.flatnonzero(z))
    for v in I:
        out = sorted(u for u in nbr[v] if u not in I)
        for u, w in itertools.combinations(out, 2):
            if _independent(nbr, (I - {v}) | {u, w}):
                return True
    return False


def _maximal_independent(g, z):
    nbr = _adj_sets(g)
    I = set(int(v) for v in np.flatnonzero(z))
    return _independent(nbr, I) and all(nbr[v] & I for v in range(g.n) if v not in I)


def _cut(g, s):
    return int(discrete.evaluate_cut(g, np.asarray(s).reshape(-1, 1))[0])


def _one_flip_repairable(g, s):
    base = _cut(g, s)
    for v in range(g.n):
        t = s.copy()
        t[v] = -t[v]
        if _cut(g, t) > base:
            return True
    return False


def _two_flip_repairable(g, s):
    """Def. 2.5 by brute force over the cut edges."""
    base = _cut(g, s)
    u, v, _ = g.edges()
    for a, b in zip(u, v):
        if s[a] != s[b]:
            t = s.copy()
            t[a], t[b] = -t[a], -t[b]
            if _cut(g, t) > base:
                return True
    return False


def _mis_graphs():
    return [graphs.erdos_renyi(14, 0.3, 4100 + i) for i in range(6)] + [graphs.star(6), graphs.path(7),
                                                                        graphs.cycle(9)]


def test_one_two_swap_worked_example_path():
    """Def. 2.3 on the path a - b - c: I = {b} is maximal and repairable;
    the swap gives {a, c}."""
    g = graphs.path(3)
    z = np.array([[0], [1], [0]], dtype=np.int8)
    assert _maximal_independent(g, z[:, 0]) and _swap_repairable(g, z[:, 0])
    out, moves = discrete.pair_search("mis", g, z, 5, np.arange(1), 0)
    assert out[:, 0].tolist() == [1, 0, 1] and moves.tolist() == [1]


def test_one_two_swap_star_ends_at_all_leaves():
    """Star with k leaves from {centre}: one swap inserts two leaves, the
    others become free and the 1-flip search adds them: size k."""
    k = 9
    g = graphs.star(k)
    z = np.zeros((k + 1, 3), dtype=np.int8)
    z[0] = 1
    out, moves = discrete.pair_search("mis", g, z, 8, np.arange(3), 2)
    assert np.all(out[0] == 0) and np.all(out[1:] == 1) and moves.tolist() == [1, 1, 1]


@pytest.mark.parametrize("gi", range(9))
def test_one_two_swap_ends_maximal_and_not_repairable(gi):
    g = _mis_graphs()[gi]
    rng = np.random.default_rng(4200 + gi)
    Z = (rng.random((g.n, 6)) < 0.3).astype(np.int8)  # includes infeasible starts
    Z[:, 0] = 0
    out, moves = discrete.pair_search("mis", g, Z, 9, np.arange(6), 1)
    ls, _ = discrete.local_search("mis", g, Z, 9, np.arange(6), 1)
    for b in range(6):
        assert _maximal_independent(g, out[:, b])
        assert not _swap_repairable(g, out[:, b])
        # the search starts from the 1-flip result and every swap adds one
        assert out[:, b].sum() >= ls[:, b].sum() + moves[b]


def test_one_two_swap_parallel_moves_add():
    """On a maximal independent set, the moves of one parallel iteration are
    each valid alone and together give |I| + (number of moves)."""
    hits = 0
    for seed in range(20):
        g = graphs.erdos_renyi(40, 0.12, 4300 + seed)
        z0, _ = discrete.local_search("mis", g, np.zeros((g.n, 1), np.int8), seed, np.arange(1), 0)
        z = z0[:, 0].astype(np.int64)
        m = discrete.neighbour_counts(g, z.reshape(-1, 1))[:, 0]
        prio = np.random.default_rng(seed).integers(0, 1 << 32, g.n)
        app = discrete.swap_iteration_mis(g, z, m, prio)
        nbr = _adj_sets(g)
        I = set(int(v) for v in np.flatnonzero(z))
        J = set(I)
        for v, u, w in app:
            assert v in I and u in nbr[v] and w in nbr[v] and u not in I and w not in I
            assert _independent(nbr, (I - {v}) | {u, w})
            J = (J - {v}) | {u, w}
        assert _independent(nbr, J) and len(J) == len(I) + len(app)
        hits += bool(app)
    assert hits > 0


def test_one_two_flip_worked_example_c4():
    """C4 with s = (+, +, -, -): every single flip keeps the cut at 2, the
    2-flip of the cut edge (1, 2) gives the alternating cut of 4."""
    g = graphs.cycle(4)
    s = np.array([1, 1, -1, -1], dtype=np.int8)
    assert not _one_flip_repairable(g, s) and _two_flip_repairable(g, s)
    out, moves = discrete.pair_search("maxcut", g, s.reshape(-1, 1), 3, np.arange(1), 0)
    assert _cut(g, out[:, 0]) == 4 and moves[0] == 1


def _cut_graphs():
    return [graphs.erdos_renyi(16, 0.3, 4400 + i) for i in range(4)] + [
        graphs.with_weights(graphs.erdos_renyi(14, 0.35, 4410), 4411, values=(-2, -1, 1, 3)),
        graphs.torus_pm1(4, 4412), graphs.cycle(8), graphs.random_regular(12, 4, 4413)]


@pytest.mark.parametrize("gi", range(8))
def test_one_two_flip_ends_at_a_one_and_two_flip_optimum(gi):
    g = _cut_graphs()[gi]
    rng = np.random.default_rng(4500 + gi)
    S = np.where(rng.random((g.n, 6)) < 0.5, 1, -1).astype(np.int8)
    out, moves = discrete.pair_search("maxcut", g, S, 4, np.arange(6), 3)
    ls, _ = discrete.local_search("maxcut", g, S, 4, np.arange(6), 3)
    for b in range(6):
        assert not _one_flip_repairable(g, out[:, b].astype(np.int64))
        assert not _two_flip_repairable(g, out[:, b].astype(np.int64))
        assert _cut(g, out[:, b]) >= _cut(g, ls[:, b]) + moves[b]


def test_one_two_flip_parallel_moves_add():
    """At a 1-flip optimum, the pairs of one parallel iteration are cut edges
    whose flips, applied together, change the cut by the sum of their
    individual brute-force gains, each positive."""
    hits = 0
    for seed in range(20):
        g = graphs.erdos_renyi(40, 0.1, 4600 + seed)
        s0, _ = discrete.local_search("maxcut", g, np.ones((g.n, 1), np.int8), seed, np.arange(1), 0)
        s = s0[:, 0].astype(np.int64)
        t = discrete.neighbour_counts(g, s.reshape(-1, 1))[:, 0]
        prio = np.random.default_rng(seed).integers(0, 1 << 32, g.n)
        app = discrete.flip2_iteration_cut(g, s, t, prio)
        base = _cut(g, s)
        total, r = 0, s.copy()
        for v, u in app:
            assert s[v] != s[u]
            q = s.copy()
            q[v], q[u] = -q[v], -q[u]
            gain = _cut(g, q) - base
            assert gain > 0
            total += gain
            r[v], r[u] = -r[v], -r[u]
        assert _cut(g, r) == base + total
        hits += bool(app)
    assert hits > 0


def test_two_flip_never_applies_on_odd_regular_graphs():
    """On a d-regular graph with d odd, every 1-flip gain at a 1-flip
    optimum is odd and <= -1, so no pair gains: the search equals the
    1-flip search."""
    g = graphs.random_regular(60, 3, 4700)
    S = np.where(np.random.default_rng(1).random((60, 8)) < 0.5, 1, -1).astype(np.int8)
    out, moves = discrete.pair_search("maxcut", g, S, 2, np.arange(8), 0)
    ls, _ = discrete.local_search("maxcut", g, S, 2, np.arange(8), 0)
    assert np.array_equal(out, ls) and np.all(moves == 0)


@pytest.mark.parametrize("kind", ["mis", "maxcut"])
def test_solver_final_search_ends_at_pair_optima(kind):
    """Alg. 1 / Alg. 2: the search after the reset loop leaves incumbents
    that no 1-flip, (1,2)-swap or 2-flip improves, never worse than
    without it."""
    from oracle import solver
    g = graphs.erdos_renyi(18, 0.25, 4800)
    kw = dict(batch=5, steps_per_round=30, rounds=3, alpha=0.05, seed=48)
    plain = solver.solve(kind, g, solver.Params(**kw))
    fin = solver.solve(kind, g, solver.Params(final_search=True, **kw))
    assert np.all(fin["traj_best_value"] >= plain["traj_best_value"])
    for b in range(5):
        z = fin["traj_best_x"][:, b]
        if kind == "mis":
            assert _maximal_independent(g, z) and not _swap_repairable(g, z)
        else:
            s = z.astype(np.int64)
            assert not _one_flip_repairable(g, s) and not _two_flip_repairable(g, s)


def test_two_flip_numpy_form_equals_loop_form():
    for seed in range(12):
        g = graphs.erdos_renyi(60, 0.08, 4950 + seed)
        if seed % 3 == 1:
            g = graphs.with_weights(g, 4970 + seed, values=(-2, -1, 1, 3))
        if seed % 3 == 2:
            g = graphs.torus_pm1(7, 4990 + seed)
        rng = np.random.default_rng(seed)
        s = np.where(rng.random(g.n) < 0.5, 1, -1).astype(np.int64)
        s = discrete.local_search("maxcut", g, s.reshape(-1, 1), seed, np.arange(1), 0)[0][:, 0].astype(np.int64)
        t = discrete.neighbour_counts(g, s.reshape(-1, 1))[:, 0]
        prio = rng.integers(0, 1 << 32, g.n)
        prio[: g.n // 3] = prio[0]  # ties in the hash
        a = discrete.flip2_iteration_cut(g, s, t, prio)
        b = discrete.flip2_iteration_cut_np(g, s, t, prio)
        assert sorted(a) == sorted(b)
