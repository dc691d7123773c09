"""The optional early exit of the schedule (a trajectory stops stepping for
the rest of a round once its rounded point is a fixed point of the projected
step), pinned on the CPU oracle."""
import itertools

import numpy as np
import pytest

from synth import graphs
from oracle import objectives as obj, discrete, solver


def _all_spins(n):
    return np.array(list(itertools.product([-1, 1], repeat=n)), dtype=np.int8).T  # [n][2^n]


@pytest.mark.parametrize("seed", range(4))
def test_cut_fixed_points_are_one_flip_optima(seed):
    """Gain identity (proof of Prop. 3.4): flipping v changes the cut by
    s_v (A s)_v.  A binary s that the projected f_B step keeps is a 1-flip
    local optimum, and every strict 1-flip optimum is kept."""
    g = graphs.with_weights(graphs.erdos_renyi(9, 0.45, 700 + seed), 701 + seed)
    S = _all_spins(g.n)
    fixed = discrete.is_pga_fixed_cut(g, S, 1e-3, alpha=0.01)
    gain = discrete.gains(obj.MAXCUT, g, S)
    assert np.all(gain[:, fixed] <= 0)
    assert np.all(fixed[np.all(gain < 0, axis=0)])
    # independent of the (positive) step size
    assert np.array_equal(fixed, discrete.is_pga_fixed_cut(g, S, 1e-3, alpha=0.3))


def test_cut_fixed_tie_breaks_by_the_bias():
    """With s_v t_v = 0 the gradient is -lambda: only s_v = -1 stays."""
    g = graphs.path(2)
    S = np.array([[1, -1], [-1, 1]], dtype=np.int8).T  # columns (1,-1) and (-1,1) have t = -s: cut edges
    assert discrete.is_pga_fixed_cut(g, S, 1e-3, 0.01).all()
    g1 = graphs.empty(1)
    assert discrete.is_pga_fixed_cut(g1, np.array([[-1]], np.int8), 1e-3, 0.01)[0]
    assert not discrete.is_pga_fixed_cut(g1, np.array([[1]], np.int8), 1e-3, 0.01)[0]


@pytest.mark.parametrize("kind", [obj.MIS, obj.MAXCUT])
def test_early_exit_stops_at_fixed_points(kind):
    g = graphs.erdos_renyi(60, 0.08, 710)
    alpha = 0.05 if kind == obj.MIS else 0.2  # f_B iterates reach binary fixed points slowly
    base = dict(batch=12, steps_per_round=120, rounds=3, alpha=alpha, seed=711, rho=0.1)
    param = 2.0 if kind == obj.MIS else 1e-3
    st = {}
    tr = []
    p = solver.Params(check_every=10, **base)
    vals, zb = solver.solve_graph(kind, g, p, stats=st, trace=tr)
    steps = st["steps"]
    # someone stopped early, nobody ran more than the schedule, whole chunks only
    assert steps.min() < 3 * 120 and steps.max() <= 3 * 120
    # a check past the schedule's end never fires: same result as no check
    q = solver.Params(check_every=500, **base)
    st2 = {}
    v2, z2 = solver.solve_graph(kind, g, q, stats=st2)
    r2 = solver.solve_graph(kind, g, solver.Params(**base))
    assert np.array_equal(v2, r2[0]) and np.array_equal(z2, r2[1])
    assert np.all(st2["steps"] == 3 * 120)
    # one round, checked every step: the stopping iterate rounds to a fixed point
    p1 = solver.Params(check_every=1, **dict(base, rounds=1, rho=0.0))
    st1 = {}
    solver.solve_graph(kind, g, p1, stats=st1)
    s1 = st1["steps"]
    from oracle import pga
    X = pga.init_uniform(kind, g.n, np.arange(12), 711)
    for c in range(12):
        x = X[:, [c]]
        for _ in range(s1[c]):
            x, _ = pga.step32(g, x, kind, alpha, param)
        if s1[c] < 120:
            assert discrete.is_pga_fixed(kind, g, discrete.round_x(kind, x), param, alpha)[0]
            # and it was not fixed one step earlier
            y = X[:, [c]]
            for _ in range(s1[c] - 1):
                y, _ = pga.step32(g, y, kind, alpha, param)
            assert not discrete.is_pga_fixed(kind, g, discrete.round_x(kind, y), param, alpha)[0]


def test_mis_early_exit_points_are_maximal_independent_sets():
    g = graphs.erdos_renyi(40, 0.1, 720)
    p = solver.Params(batch=16, steps_per_round=200, rounds=1, alpha=0.05, seed=721, check_every=5,
                      local_search=False)
    st = {}
    vals, zb = solver.solve_graph(obj.MIS, g, p, stats=st)
    stopped = st["steps"] < 200
    assert stopped.any()
    assert np.all(discrete.is_maximal_independent(g, zb)[stopped])
