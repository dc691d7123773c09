"""The batched mutation-guided search (Alg. 1 / Alg. 2 run for B independent
trajectories, the batch form of Alg. 3 / Alg. 4 without the top-K pool).

Round r = 0 .. rounds-1 of trajectory t = g*B + b:
  * r = 0 starts from x0 (given, or drawn by the initialisation rule);
    r > 0 starts from the incumbent with the reset set R zeroed (Sec. 4;
    Alg. 1 / Alg. 2 reset loop), momentum cleared;
  * ``steps_per_round`` PGA steps (float32 replay, or float64); with
    ``check_every`` = c > 0, after every c steps of a round (before its
    end) a trajectory whose rounded point is a fixed point of the projected
    step (the checker of Eq. (8) for MIS, its f_B analogue for MaxCut)
    stops stepping for the rest of the round (Alg. 1 / Alg. 2 run PGA
    until a MIS is detected / until convergence);
  * threshold rounding (Sec. 3);
  * optional 1-flip local search (parallel rule, ``discrete.local_search``);
  * exact evaluation; accept iff strictly better than the incumbent
    (Sec. 4), round 0 always initialises the incumbent.
With ``final_search`` the paper's own search (OneTwoSwap / OneTwoFlip,
``discrete.pair_search``) runs at the end of every outer iteration (below;
without ``restart_every`` the one iteration ends after the last round),
with round index ``rounds + j`` for outer iteration j: on every incumbent,
replacing it when strictly better, so the reset rounds of the next
iteration start from the searched set (Alg. 1 / Alg. 2, the local search
closing each pass of the outer loop).
With ``restart_every`` = R > 0 the outer loop of Alg. 1-4 (a fresh
initialisation followed by reset rounds, repeated while time remains) is
unrolled into the rounds: every
round r > 0 with r % R == 0 starts from a fresh initial point (the
initialisation rule, start index r // R) instead of a reset; acceptance,
incumbents and the pool carry over.
With ``pool_k`` = K > 0 the graph's trajectories share the pmQO pool of
Alg. 3 / Alg. 4: after every round the pool becomes the top K distinct
solutions of the pool and the round's candidates (``discrete.pool_update``),
and a round r > 0 restarts trajectory t from pool slot
``discrete.pool_bases`` (its own incumbent while the pool is empty).  The
graph also keeps its best set I_sol / S_sol, replaced by the best pool
member after every round when that is strictly better; it is the answer.
``final_search`` then leaves the pool alone and at the end of every outer
iteration searches I_sol alone (MIS, Alg. 3, trajectory id g K) or every
pool member (MaxCut, Alg. 4, trajectory ids g K + slot, offered to S_sol
in slot order, each taken when strictly better).
The answer of graph g is the best incumbent over its B trajectories, ties
to the lowest b.
``rounds_run`` = q (1 <= q <= rounds) stands for a time budget that runs out
after q rounds (the outer loop of Alg. 1-4 repeats while time remains): the
later rounds never start, the pass they cut short still ends with the
search, and the searches keep their round indices ``rounds + j``.
Test infrastructure only.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import discrete
from . import objectives as obj
from . import pga


@dataclasses.dataclass
class Params:
    batch: int
    steps_per_round: int
    rounds: int
    alpha: float
    seed: int
    gamma: float = 2.0
    lam: float = 1e-3
    mu: float = 0.0
    rho: float = 0.05
    reset_mode: str = "zero"
    local_search: bool = True
    init_mode: str = "uniform"
    init_sigma: float = 0.0
    check_every: int = 0
    final_search: bool = False
    pool_k: int = 0
    restart_every: int = 0
    rounds_run: int | None = None


def solve_graph(kind, graph, p: Params, graph_index=0, x0=None, precision="fp32", trace=None, cols=None,
                stats=None):
    """Run the search on one graph (local indices).  Returns
    (traj_best_value int64[B], traj_best_z int8[n][B]).  Trajectories are
    independent, so ``cols`` may select a subset b of them (x0 then holds
    only those columns); the outputs hold the selected columns in order.
    ``stats`` (a dict) receives steps[B], the PGA steps each trajectory
    executed."""
    n = graph.n
    cols = np.arange(p.batch, dtype=np.int64) if cols is None else np.asarray(cols, dtype=np.int64)
    B = len(cols)
    traj = graph_index * p.batch + cols
    param = p.gamma if kind == obj.MIS else p.lam
    A = obj.adjacency(graph) if precision == "fp64" else None
    k = discrete.reset_count(p.rho, n)
    best = np.full(B, np.iinfo(np.int64).min, dtype=np.int64)
    zbest = np.zeros((n, B), dtype=np.int8)
    steps = np.zeros(B, dtype=np.int64)
    K = p.pool_k
    if K:
        assert B == p.batch, "the pool couples all trajectories of a graph"
    pool_val, pool_z = np.zeros(0, dtype=np.int64), np.zeros((n, 0), dtype=np.int8)
    NONE = int(np.iinfo(np.int64).min)
    sol_val, sol_z = NONE, np.zeros(n, dtype=np.int8)  # I_sol / S_sol of the pool mode
    last = (p.rounds if p.rounds_run is None else p.rounds_run) - 1
    assert 0 <= last < p.rounds
    for r in range(last + 1):
        fresh = r > 0 and p.restart_every > 0 and r % p.restart_every == 0
        start = r // p.restart_every if fresh else 0
        if r == 0 and x0 is not None:
            X = np.asarray(x0, dtype=np.float32)
        elif r == 0 or fresh:
            if p.init_mode == "uniform":
                X = pga.init_uniform(kind, n, traj, p.seed, start)
            else:
                X = pga.init_degree(kind, graph.degrees(), traj, p.seed, p.init_sigma, start).astype(np.float32)
        else:
            mask = discrete.reset_set(n, k, p.seed, traj, r)
            base = zbest
            if K and len(pool_val):
                base = pool_z[:, discrete.pool_bases(p.seed, traj, r, len(pool_val))]
            X = discrete.reset_apply(kind, base, mask, p.reset_mode)
        V = None
        active = np.ones(B, dtype=bool)
        for st in range(p.steps_per_round):
            if not active.any():
                break
            if precision == "fp32":
                Xn, Vn = pga.step32(graph, X, kind, p.alpha, param, p.mu, V)
            else:
                Xn, Vn = pga.step64(X, A, kind, p.alpha, param, p.mu, V)
            # stopped trajectories keep their iterate (and momentum)
            X = np.where(active[None, :], Xn, X)
            V = Vn if V is None or Vn is None else np.where(active[None, :], Vn, V)
            steps += active
            done = st + 1
            if p.check_every > 0 and done % p.check_every == 0 and done < p.steps_per_round:
                fixed = discrete.is_pga_fixed(kind, graph, discrete.round_x(kind, X), param, p.alpha)
                active &= ~fixed
        Z = discrete.round_x(kind, X)
        if p.local_search:
            Z, _ = discrete.local_search(kind, graph, Z, p.seed, traj, r)
        val = discrete.value(kind, graph, Z)
        take = (val > best) if r else np.ones(B, dtype=bool)
        best = np.where(take, val, best)
        zbest[:, take] = Z[:, take]
        if K:
            pool_val, pool_z = discrete.pool_update(kind, pool_val, pool_z, val, Z, K)
            # Alg. 3 / Alg. 4: the best set follows the pool's best member
            if len(pool_val) and pool_val[0] > sol_val:
                sol_val, sol_z = int(pool_val[0]), pool_z[:, 0].copy()
        if trace is not None:
            trace.append(dict(round=r, value=val.copy(), best=best.copy()))
        # the outer iteration ends after the last of its R rounds, or after
        # the last round of the run
        ends = (p.restart_every > 0 and (r + 1) % p.restart_every == 0) or r == last
        if p.final_search and ends:
            rnd = p.rounds + (r // p.restart_every if p.restart_every > 0 else 0)
            if not K:
                # Alg. 1 / Alg. 2: every chain's own best set
                Zs, _ = discrete.pair_search(kind, graph, zbest, p.seed, traj, rnd)
                vs = discrete.value(kind, graph, Zs)
                take = vs > best
                best = np.where(take, vs, best)
                zbest[:, take] = Zs[:, take]
            elif kind == obj.MIS:
                # Alg. 3: I_sol alone
                if sol_val != NONE:
                    Zs, _ = discrete.pair_search(kind, graph, sol_z[:, None], p.seed,
                                                 np.array([graph_index * K]), rnd)
                    vs = int(discrete.value(kind, graph, Zs)[0])
                    if vs > sol_val:
                        sol_val, sol_z = vs, Zs[:, 0].copy()
            elif len(pool_val):
                # Alg. 4: every pool member, each offered to S_sol in slot order
                Zs, _ = discrete.pair_search(kind, graph, pool_z, p.seed,
                                             graph_index * K + np.arange(len(pool_val)), rnd)
                vs = discrete.value(kind, graph, Zs)
                for i in range(len(pool_val)):
                    if vs[i] > sol_val:
                        sol_val, sol_z = int(vs[i]), Zs[:, i].copy()
    if stats is not None:
        stats["steps"] = steps
        if K:
            stats["pool_value"], stats["pool_z"] = pool_val, pool_z
            stats["sol_value"], stats["sol_z"] = sol_val, sol_z
    return best, zbest


def solve(kind, graph, p: Params, x0=None, precision="fp32"):
    """All graphs of a batch.  Returns a dict with best_value[G],
    best_x int8[n_total], traj_best_value[G*B], traj_best_x int8[n_total][B],
    traj_steps[G*B] (PGA steps executed)."""
    G = graph.num_graphs
    offs = graph.vtx_offset
    out_vals = np.zeros(G * p.batch, dtype=np.int64)
    out_z = np.zeros((graph.n, p.batch), dtype=np.int8)
    best_value = np.zeros(G, dtype=np.int64)
    best_x = np.zeros(graph.n, dtype=np.int8)
    out_steps = np.zeros(G * p.batch, dtype=np.int64)
    # empty pool slots: value INT64_MIN, solution zeros
    pool_value = np.full(G * p.pool_k, np.iinfo(np.int64).min, dtype=np.int64)
    pool_x = np.zeros((graph.n, p.pool_k), dtype=np.int8)
    for g in range(G):
        sub = graph.subgraph(g)
        lo, hi = int(offs[g]), int(offs[g + 1])
        x0g = None if x0 is None else np.asarray(x0)[lo:hi]
        st = {}
        vals, zb = solve_graph(kind, sub, p, g, x0g, precision, stats=st)
        out_steps[g * p.batch:(g + 1) * p.batch] = st["steps"]
        out_vals[g * p.batch:(g + 1) * p.batch] = vals
        out_z[lo:hi] = zb
        if p.pool_k:
            pv, pz = st["pool_value"], st["pool_z"]
            K = p.pool_k
            pool_value[g * K:g * K + len(pv)] = pv
            pool_x[lo:hi, :len(pv)] = pz
            # the answer is I_sol / S_sol (-1 while no solution was found)
            best_value[g] = st["sol_value"] if len(pv) else -1
            best_x[lo:hi] = st["sol_z"]
            continue
        b = int(np.argmax(vals))  # first index of the maximum
        best_value[g] = vals[b]
        best_x[lo:hi] = zb[:, b]
    out = dict(best_value=best_value, best_x=best_x, traj_best_value=out_vals, traj_best_x=out_z,
               traj_steps=out_steps)
    if p.pool_k:
        out["pool_value"], out["pool_x"] = pool_value, pool_x
    return out
