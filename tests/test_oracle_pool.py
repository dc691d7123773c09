"""Pins of the oracle's pmQO pool (Alg. 3 / Alg. 4): the hash generator,
TopK of a set union checked by exact byte comparison, base sampling, and
the solver's pool mode.  CPU only."""
import numpy as np
import pytest

from synth import graphs
from oracle import discrete, philox, solver


def test_splitmix64_reference_sequence():
    """The first outputs of SplitMix64 seeded with 0 (the published
    generator; state advances by the golden gamma)."""
    g = 0x9E3779B97F4A7C15
    states = np.array([0, g, (2 * g) % (1 << 64)], dtype=np.uint64)
    out = [int(v) for v in discrete.splitmix64(states)]
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def _topk_exact(kind, pool_val, pool_z, val, Z, K):
    """TopK of the union by exact comparison of the solution bytes."""
    items = [(int(pool_val[i]), i, pool_z[:, i].tobytes()) for i in range(len(pool_val))]
    items += [(int(val[b]), len(pool_val) + b, Z[:, b].tobytes()) for b in range(Z.shape[1])
              if not (kind == "mis" and val[b] < 0)]
    best = {}
    for v, src, zb in items:  # keep the earliest source of every distinct solution
        if zb not in best or (-v, src) < (-best[zb][0], best[zb][1]):
            best[zb] = (v, src)
    ranked = sorted(((v, src, zb) for zb, (v, src) in best.items()), key=lambda t: (-t[0], t[1]))[:K]
    return [t[0] for t in ranked], [np.frombuffer(t[2], dtype=np.int8) for t in ranked]


@pytest.mark.parametrize("kind", ["mis", "maxcut"])
def test_pool_update_is_topk_of_the_union(kind):
    rng = np.random.default_rng(7)
    n = 12
    for trial in range(40):
        K = int(rng.integers(1, 6))
        base = (rng.random((n, 5)) < 0.5).astype(np.int8)
        if kind == "maxcut":
            base = np.where(base > 0, 1, -1).astype(np.int8)
        # candidates drawn from few distinct vectors, so duplicates are common
        Z = base[:, rng.integers(0, 5, 9)]
        val = np.array([int(np.abs(Z[:, b]).sum() % 4) - (1 if kind == "mis" and b % 4 == 3 else 0)
                        for b in range(9)], dtype=np.int64)
        # the same solution always carries the same value
        key = {Z[:, b].tobytes(): val[b] for b in range(9)}
        val = np.array([key[Z[:, b].tobytes()] for b in range(9)], dtype=np.int64)
        pv, pz = discrete.pool_update(kind, np.zeros(0, np.int64), np.zeros((n, 0), np.int8), val[:4], Z[:, :4], K)
        pv2, pz2 = discrete.pool_update(kind, pv, pz, val[4:], Z[:, 4:], K)
        ev, ez = _topk_exact(kind, pv, pz, val[4:], Z[:, 4:], K)
        assert pv2.tolist() == ev
        assert all(np.array_equal(pz2[:, i], ez[i]) for i in range(len(ev)))


def test_pool_bases_uniform_over_slots():
    size = 5
    b = discrete.pool_bases(3, np.arange(20000), 4, size)
    counts = np.bincount(b, minlength=size)
    exp = 20000 / size
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert b.min() >= 0 and b.max() < size and chi2 < 20.5  # 4 dof, p ~ 4e-4


@pytest.mark.parametrize("kind", ["mis", "maxcut"])
def test_solver_pool_mode(kind):
    g = graphs.concat([graphs.erdos_renyi(40, 0.12, 5100), graphs.erdos_renyi(30, 0.15, 5101)])
    K, B = 3, 5
    p = solver.Params(batch=B, steps_per_round=25, rounds=4, alpha=0.05, seed=51, pool_k=K)
    r = solver.solve(kind, g, p)
    for gi in range(g.num_graphs):
        lo, hi = g.vtx_offset[gi], g.vtx_offset[gi + 1]
        sub = g.subgraph(gi)
        pv = r["pool_value"][gi * K:(gi + 1) * K]
        filled = pv > np.iinfo(np.int64).min
        pz = r["pool_x"][lo:hi][:, filled]
        # sorted, distinct, and each value is its solution's value
        assert np.all(np.diff(pv[filled]) <= 0)
        assert len({pz[:, i].tobytes() for i in range(pz.shape[1])}) == pz.shape[1]
        assert np.array_equal(discrete.value(kind, sub, pz), pv[filled])
        # the answer is the best pool member, never below any incumbent
        assert r["best_value"][gi] == pv[filled].max()
        assert r["best_value"][gi] >= r["traj_best_value"][gi * B:(gi + 1) * B].max()


def test_pool_of_one_restarts_everyone_from_the_best():
    """K = 1: every round restarts every trajectory from the single best
    solution so far."""
    g = graphs.erdos_renyi(50, 0.1, 5200)
    trace = []
    p = solver.Params(batch=4, steps_per_round=20, rounds=3, alpha=0.05, seed=52, pool_k=1)
    solver.solve_graph("mis", g, p, trace=trace)
    assert np.all(discrete.pool_bases(52, np.arange(4), 2, 1) == 0)
    best_so_far = max(int(t["value"].max()) for t in trace)
    r = solver.solve("mis", g, p)
    assert r["best_value"][0] == best_so_far


def test_restarts_unroll_the_outer_loop():
    """restart_every = R: rounds 0, R, 2R, ... start from fresh points (start
    index r // R); a restart round with no reset rounds between is the same
    as an independent solve from that start, and incumbents carry over."""
    from oracle import pga
    g = graphs.erdos_renyi(60, 0.1, 5300)
    # no local search: its priorities depend on the round index
    kw = dict(batch=4, steps_per_round=30, alpha=0.05, seed=53, local_search=False)
    trace = []
    solver.solve_graph("mis", g, solver.Params(rounds=6, restart_every=2, **kw), trace=trace)
    # round 2 is the second start: its candidate equals round 0 of a solve
    # started from init start 1
    x1 = pga.init_uniform("mis", g.n, np.arange(4), 53, start=1)
    t2 = []
    solver.solve_graph("mis", g, solver.Params(rounds=1, **kw), x0=x1, trace=t2)
    assert np.array_equal(trace[2]["value"], t2[0]["value"])
    # incumbents never decrease across restarts
    bests = np.array([t["best"] for t in trace])
    assert np.all(np.diff(bests, axis=0) >= 0)
    # the fresh starts differ from the first one
    assert not np.array_equal(x1, pga.init_uniform("mis", g.n, np.arange(4), 53))
