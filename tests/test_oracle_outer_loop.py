"""Pins of the oracle's outer loop with the paper's own search (Alg. 1-4):
the search closes every pass of the outer loop, so the reset rounds of the
next pass start from the searched best set (Alg. 1 / Alg. 2); in pool mode
it improves I_sol / S_sol and leaves the pool alone (Alg. 3 / Alg. 4).

The worked examples use zero PGA steps and rho = 0, so a reset round
reproduces its base exactly and every candidate value follows by hand from
the graph: on the path a - b - c the maximal independent sets are {b}
(size 1) and {a, c} (size 2, what one (1,2)-swap makes of {b}); on C4 the
1-flip optima are the two alternating cuts (4) and the splits into two
adjacent pairs (2, which one 2-flip turns into an alternating cut).  The
run seeds are chosen so that the fresh start of the second pass lands on
the worse optimum; that is asserted too.  CPU only."""
import numpy as np
import pytest

from synth import graphs
from oracle import discrete, solver

from test_oracle_pair_search import (_maximal_independent, _one_flip_repairable, _swap_repairable,
                                     _two_flip_repairable)

MIN = np.iinfo(np.int64).min


def _params(**kw):
    base = dict(batch=1, steps_per_round=0, rounds=4, alpha=0.05, rho=0.0, final_search=True, restart_every=2)
    base.update(kw)
    return solver.Params(**base)


def test_mis_search_of_each_pass_seeds_the_next_resets():
    """Alg. 1: rounds 0-1 hold {b}; the search after round 1 makes it
    {a, c}; round 2 (a fresh start) finds {b} again and is not taken; round 3
    resets from the searched {a, c}, so its candidate has size 2.  With the
    search only after the last round, round 3 would restart from {b}."""
    g = graphs.path(3)
    x0 = np.array([[0.2], [0.9], [0.2]], dtype=np.float32)
    trace = []
    best, zb = solver.solve_graph("mis", g, _params(seed=3), x0=x0, trace=trace)
    assert [int(t["value"][0]) for t in trace] == [1, 1, 1, 2]
    assert [int(t["best"][0]) for t in trace] == [1, 1, 2, 2]  # round 2 enters with the searched set
    assert best.tolist() == [2] and zb[:, 0].tolist() == [1, 0, 1]


def test_maxcut_search_of_each_pass_seeds_the_next_resets():
    """Alg. 2 on C4: s = (+, +, -, -) cuts 2; the search after round 1
    makes it alternating (4); round 2's fresh start cuts 2; round 3 resets
    from the alternating cut."""
    g = graphs.cycle(4)
    x0 = np.array([[0.5], [0.5], [-0.5], [-0.5]], dtype=np.float32)
    trace = []
    best, zb = solver.solve_graph("maxcut", g, _params(seed=1), x0=x0, trace=trace)
    assert [int(t["value"][0]) for t in trace] == [2, 2, 2, 4]
    assert best.tolist() == [4]
    s = zb[:, 0].astype(np.int64)
    assert all(s[i] != s[(i + 1) % 4] for i in range(4))


def test_mis_pool_searches_i_sol_and_leaves_the_pool():
    """Alg. 3 on the path: both trajectories find {b}, the pool holds it
    once and I_sol = {b}; the search after the last round makes I_sol
    {a, c} (the answer) while the pool, the trajectories' incumbents and
    the reset bases keep {b}."""
    g = graphs.path(3)
    x0 = np.tile(np.array([[0.2], [0.9], [0.2]], dtype=np.float32), (1, 2))
    r = solver.solve("mis", g, _params(batch=2, pool_k=2, rounds=2, restart_every=0, seed=3), x0=x0)
    assert r["best_value"].tolist() == [2] and r["best_x"].tolist() == [1, 0, 1]
    assert r["pool_value"].tolist() == [1, MIN]
    assert r["pool_x"][:, 0].tolist() == [0, 1, 0]
    assert r["traj_best_value"].tolist() == [1, 1]


def test_mis_pool_resets_from_the_pool_not_from_i_sol():
    """Alg. 3 with two passes: after the first search I_sol = {a, c}, but
    the second pass samples its bases from the pool, which still holds {b}
    only (the fresh start finds {b} in both trajectories), so round 3's
    candidates have size 1."""
    g = graphs.path(3)
    x0 = np.tile(np.array([[0.2], [0.9], [0.2]], dtype=np.float32), (1, 2))
    trace = []
    st = {}
    solver.solve_graph("mis", g, _params(batch=2, pool_k=2, seed=5), x0=x0, trace=trace, stats=st)
    assert [t["value"].tolist() for t in trace] == [[1, 1], [1, 1], [1, 1], [1, 1]]
    assert st["sol_value"] == 2 and st["sol_z"].tolist() == [1, 0, 1]
    assert st["pool_value"].tolist() == [1]


def test_maxcut_pool_searches_every_member_for_s_sol():
    """Alg. 4 on C4: the two trajectories give the two pair splits
    (+, +, -, -) and (+, -, -, +), both cut 2 and both in the pool; the
    search turns each into an alternating cut of 4; S_sol takes the first
    (slot 0's) and the pool keeps its cuts of 2."""
    g = graphs.cycle(4)
    x0 = np.array([[0.5, 0.5], [0.5, -0.5], [-0.5, -0.5], [-0.5, 0.5]], dtype=np.float32)
    r = solver.solve("maxcut", g, _params(batch=2, pool_k=2, rounds=2, restart_every=0, seed=1), x0=x0)
    assert r["pool_value"].tolist() == [2, 2]
    assert r["pool_x"][:, 0].tolist() == [1, 1, -1, -1] and r["pool_x"][:, 1].tolist() == [1, -1, -1, 1]
    assert r["best_value"].tolist() == [4]
    s = r["best_x"].astype(np.int64)
    assert all(s[i] != s[(i + 1) % 4] for i in range(4))
    # slot 0's searched set, trajectory id 0, round index rounds + 0
    z0, _ = discrete.pair_search("maxcut", g, r["pool_x"][:, :1], 1, np.array([0]), 2)
    assert np.array_equal(z0[:, 0], r["best_x"])


@pytest.mark.parametrize("kind", ["mis", "maxcut"])
@pytest.mark.parametrize("pool_k", [0, 3])
def test_answers_are_pair_optimal_after_every_pass(kind, pool_k):
    """Whatever the placement, the answer after the last pass is a point no
    1-flip, (1,2)-swap or 2-flip improves (checked by brute force over the
    moves of Def. 2.3 / 2.5), never below the search-free answer; without
    the pool so is every incumbent."""
    g = graphs.erdos_renyi(18, 0.25, 4810)
    kw = dict(batch=4, steps_per_round=25, rounds=5, alpha=0.05, seed=49, restart_every=2, pool_k=pool_k,
              rho=0.1)
    plain = solver.solve(kind, g, solver.Params(**kw))
    fin = solver.solve(kind, g, solver.Params(final_search=True, **kw))
    assert fin["best_value"][0] >= plain["best_value"][0]
    cols = [fin["best_x"]] + ([] if pool_k else [fin["traj_best_x"][:, b] for b in range(4)])
    for z in cols:
        if kind == "mis":
            assert _maximal_independent(g, z) and not _swap_repairable(g, z)
        else:
            s = z.astype(np.int64)
            assert not _one_flip_repairable(g, s) and not _two_flip_repairable(g, s)
    if pool_k:
        # the pool is the same with and without the search of Alg. 3 / 4
        assert np.array_equal(fin["pool_value"], plain["pool_value"])
        assert np.array_equal(fin["pool_x"], plain["pool_x"])


def test_budget_cut_runs_the_first_rounds_and_still_searches_the_cut_pass():
    """rounds_run = q stands for a time budget that runs out after q rounds:
    without the search the run is a q-round run; with it the pass the budget
    cut short still ends with the search (on the path, round 0 holds {b}
    and the search makes it {a, c})."""
    g = graphs.path(3)
    x0 = np.array([[0.2], [0.9], [0.2]], dtype=np.float32)
    for q in (1, 2, 3):
        cut = solver.solve_graph("mis", g, _params(seed=3, final_search=False, rounds_run=q), x0=x0)
        short = solver.solve_graph("mis", g, _params(seed=3, final_search=False, rounds=q), x0=x0)
        assert np.array_equal(cut[0], short[0]) and np.array_equal(cut[1], short[1])
    trace = []
    best, zb = solver.solve_graph("mis", g, _params(seed=3, rounds_run=1), x0=x0, trace=trace)
    assert len(trace) == 1 and int(trace[0]["value"][0]) == 1
    assert best.tolist() == [2] and zb[:, 0].tolist() == [1, 0, 1]
    with pytest.raises(AssertionError):
        solver.solve_graph("mis", g, _params(seed=3, rounds_run=5), x0=x0)
