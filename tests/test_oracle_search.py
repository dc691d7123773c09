"""Pins of the oracle's step replay, local search, reset, solver and
adjoint.  CPU only."""
import numpy as np
import pytest

from synth import graphs, arrays
from oracle import philox, objectives as obj, pga, discrete, solver, brute


# --------------------------------------------------------------------------
# float32 replay against float64 truth
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", [obj.MIS, obj.MAXCUT])
@pytest.mark.parametrize("weighted", [False, True])
def test_step32_close_to_step64(kind, weighted):
    g = graphs.erdos_renyi(300, 0.05, 201)
    if weighted:
        if kind == obj.MIS:
            pytest.skip("MIS is unweighted")
        g = graphs.with_weights(g, 202)
    lo, hi = obj.box(kind)
    X = arrays.uniform((300, 9), lo, hi, 203)
    param = 2.0 if kind == obj.MIS else 1e-3
    A = obj.adjacency(g)
    for mu in (0.0, 0.7):
        V = arrays.uniform((300, 9), -1, 1, 204) if mu else None
        x32, v32 = pga.step32(g, X, kind, 0.01, param, mu, V)
        x64, v64 = pga.step64(X.astype(np.float64), A, kind, 0.01, param, mu,
                              None if V is None else V.astype(np.float64))
        rel = np.abs(x32 - x64).max() / max(1.0, np.abs(x64).max())
        assert rel <= 1e-5
        g32 = pga.gradient32(g, X, kind, param)
        g64 = obj.gradient(kind, X.astype(np.float64), A, param)
        assert np.abs(g32 - g64).max() / max(1.0, np.abs(g64).max()) <= 1e-5


@pytest.mark.parametrize("kind", [obj.MIS, obj.MAXCUT])
def test_step32_exact_on_dyadic_inputs(kind):
    """With dyadic iterates, a power-of-two step and gamma/lambda dyadic,
    every float32 operation is exact, so the replay equals float64 bit for
    bit: a dropped term, a sign or a wrong neighbour would show."""
    g = graphs.erdos_renyi(200, 0.04, 211)
    lo, hi = obj.box(kind)
    X = (np.floor(arrays.uniform((200, 5), lo, hi, 212, np.float64) * 8) / 8).astype(np.float32)
    X = np.clip(X, lo, hi)
    param = 2.0 if kind == obj.MIS else 0.25
    A = obj.adjacency(g)
    for mu in (0.0, 0.5):
        V = (np.floor(arrays.uniform((200, 5), -1, 1, 213, np.float64) * 4) / 4).astype(np.float32) if mu else None
        x32, v32 = pga.step32(g, X, kind, 0.0625, param, mu, V)
        x64, v64 = pga.step64(X.astype(np.float64), A, kind, 0.0625, param, mu,
                              None if V is None else V.astype(np.float64))
        assert np.array_equal(x32.astype(np.float64), x64)


def test_momentum_closed_form_on_isolated_vertex():
    # isolated vertex: grad h = 1, so v_k = sum_{j<k} mu^j and x_k = x_0 + alpha sum v
    g = graphs.empty(1)
    x = np.zeros((1, 1), dtype=np.float32)
    V = None
    alpha, mu = 0.0625, 0.5
    expect = 0.0
    v = 0.0
    for _ in range(4):
        x, V = pga.step32(g, x, obj.MIS, alpha, 2.0, mu, V)
        v = mu * v + 1.0
        expect = min(1.0, expect + alpha * v)
        assert float(x[0, 0]) == expect


def test_init_uniform_and_degree():
    n, traj = 50, np.arange(7) + 3
    x = pga.init_uniform(obj.MIS, n, traj, 9)
    s = pga.init_uniform(obj.MAXCUT, n, traj, 9)
    assert x.dtype == np.float32 and np.all((x >= 0) & (x < 1))
    assert np.array_equal(s, 2 * x - 1)  # exact affine map
    g = graphs.star(9)
    d = g.degrees()
    x0 = pga.init_degree(obj.MIS, d, traj, 9, 0.0)
    assert np.allclose(x0[:, 0], 1 - d / d.max())
    c0 = pga.init_degree(obj.MAXCUT, d, traj, 9, 0.0)
    assert np.allclose(c0[:, 0], 2 * (1 - d / d.max()) - 1)
    # Box-Muller noise: mean ~0, variance ~sigma^2 over many draws
    big = pga.init_degree(obj.MAXCUT, np.full(4000, 5.0), np.arange(8), 10, 0.1)
    assert np.all(big >= -1) and np.all(big <= 1) and np.any(big == -1)
    mid = pga.init_degree(obj.MIS, np.concatenate([np.full(4000, 1.0), [2.0]]), np.arange(8), 11, 0.1)
    e = mid[:4000] - 0.5
    assert abs(e.mean()) < 0.005 and abs(e.std() - 0.1) < 0.005


# --------------------------------------------------------------------------
# local search
# --------------------------------------------------------------------------

def _brute_no_improving_flip(kind, g, Z, gamma=2.0):
    """Recompute the objective of every single flip from the definitions."""
    A = obj.adjacency(g)
    for b in range(Z.shape[1]):
        z = Z[:, b].astype(np.int64)
        if kind == obj.MAXCUT:
            base = discrete.evaluate_cut(g, z[:, None])[0]
        else:
            base = obj.h(z[:, None].astype(np.float64), A, gamma)[0]
        for v in range(g.n):
            z2 = z.copy()
            z2[v] = -z2[v] if kind == obj.MAXCUT else 1 - z2[v]
            if kind == obj.MAXCUT:
                new = discrete.evaluate_cut(g, z2[:, None])[0]
            else:
                new = obj.h(z2[:, None].astype(np.float64), A, gamma)[0]
            if new > base + 1e-9:
                return False
    return True


@pytest.mark.parametrize("kind", [obj.MIS, obj.MAXCUT])
def test_local_search_reaches_one_flip_optimum(kind):
    g = graphs.erdos_renyi(60, 0.08, 301)
    if kind == obj.MAXCUT:
        g = graphs.with_weights(g, 302)
    Z = arrays.binary01((60, 12), 303) if kind == obj.MIS else arrays.spins((60, 12), 303)
    Z2, iters = discrete.local_search(kind, g, Z, 5, np.arange(12), 1)
    assert iters > 0
    assert _brute_no_improving_flip(kind, g, Z2)
    before = discrete.value(kind, g, Z) if kind == obj.MAXCUT else None
    if kind == obj.MAXCUT:
        assert np.all(discrete.value(kind, g, Z2) >= before)
    else:
        assert np.all(discrete.is_maximal_independent(g, Z2))
        assert np.all(discrete.is_pga_fixed_mis(g, Z2, 2.0, 0.01))
    # the paper's sequential sweep also ends at a 1-flip optimum
    zs = discrete.local_search_sequential(kind, g, Z[:, 0])
    assert _brute_no_improving_flip(kind, g, zs[:, None])


def test_local_search_flips_independent_sets_with_additive_gain():
    """One parallel iteration at a time: the oracle's vectorised iteration
    equals the rule written as plain loops, F is independent, and the cut
    rises by exactly the sum of the flipped gains."""
    g = graphs.with_weights(graphs.erdos_renyi(80, 0.1, 311), 312)
    cur = arrays.spins((80, 6), 313)
    u, v, _ = g.edges()
    for _ in range(40):
        gains = discrete.gains(obj.MAXCUT, g, cur)
        if not np.any(gains > 0):
            break
        one = _one_iteration_loops(g, cur)
        got, it = discrete.local_search(obj.MAXCUT, g, cur, 5, np.arange(6), 2, stop_after=1)
        assert it == 1 and np.array_equal(got, one)
        F = one != cur
        assert not np.any(F[u] & F[v])
        delta = discrete.evaluate_cut(g, one) - discrete.evaluate_cut(g, cur)
        assert np.array_equal(delta, (gains * F).sum(0))
        cur = one
    else:
        pytest.fail("did not converge")


def _one_iteration_loops(g, Z):
    """The parallel rule for MaxCut written with plain loops."""
    nb = discrete.neighbour_counts(g, Z)
    gain = Z.astype(np.int64) * nb
    P = gain > 0
    prio = philox.vertex_u32(5, philox.PURPOSE_LS, np.arange(Z.shape[1], dtype=np.uint64)[None, :], 2,
                             np.arange(g.n, dtype=np.uint64)[:, None]).astype(np.int64)
    F = np.zeros_like(P)
    for b in range(Z.shape[1]):
        for v in range(g.n):
            if not P[v, b]:
                continue
            ok = True
            for j in range(g.row_ptr[v], g.row_ptr[v + 1]):
                uu = g.col_idx[j]
                if P[uu, b] and (gain[uu, b], prio[uu, b], -uu) > (gain[v, b], prio[v, b], -v):
                    ok = False
            F[v, b] = ok
    return np.where(F, -Z, Z).astype(np.int8)


def test_mis_local_search_repairs_and_maximalises():
    g = graphs.erdos_renyi(100, 0.1, 321)
    Z = np.ones((100, 4), dtype=np.int8)  # everything in: maximal conflicts
    Z2, _ = discrete.local_search(obj.MIS, g, Z, 1, np.arange(4), 0)
    assert np.all(discrete.is_maximal_independent(g, Z2))
    Z = np.zeros((100, 4), dtype=np.int8)
    Z2, _ = discrete.local_search(obj.MIS, g, Z, 1, np.arange(4), 0)
    assert np.all(discrete.is_maximal_independent(g, Z2))


# --------------------------------------------------------------------------
# reset
# --------------------------------------------------------------------------

def test_reset_exact_size_and_uniform():
    n, k, B = 40, 7, 4000
    mask = discrete.reset_set(n, k, 17, np.arange(B), 3)
    assert np.all(mask.sum(0) == k)
    freq = mask.sum(1)
    expected = B * k / n
    chi2 = ((freq - expected) ** 2 / expected).sum()
    # chi-square with n-1 = 39 dof: 99.9% quantile is about 72.1
    assert chi2 < 72.1
    assert discrete.reset_count(0.05, 2000) == 100
    assert discrete.reset_count(0.0, 50) == 0


def test_reset_ties_fall_to_lower_index():
    keys = np.array([[5], [3], [3], [3], [9], [1]], dtype=np.uint32)
    m = discrete.reset_set(6, 3, 0, [0], 0, keys=keys)
    assert m[:, 0].tolist() == [False, True, True, False, False, True]


def test_reset_apply_modes():
    Z = np.array([[1], [0], [1]], dtype=np.int8)
    mask = np.array([[True], [True], [False]])
    assert discrete.reset_apply(obj.MIS, Z, mask, "zero")[:, 0].tolist() == [0, 0, 1]
    assert discrete.reset_apply(obj.MIS, Z, mask, "flip")[:, 0].tolist() == [0, 1, 1]
    S = np.array([[1], [-1], [1]], dtype=np.int8)
    assert discrete.reset_apply(obj.MAXCUT, S, mask, "zero")[:, 0].tolist() == [0, 0, 1]
    assert discrete.reset_apply(obj.MAXCUT, S, mask, "flip")[:, 0].tolist() == [-1, 1, 1]


# --------------------------------------------------------------------------
# solver
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_solver_finds_brute_force_optimum_mis(seed):
    g = graphs.erdos_renyi(16, 0.25, 400 + seed)
    p = solver.Params(batch=256, steps_per_round=100, rounds=3, alpha=0.05, seed=seed, rho=0.25)
    r = solver.solve(obj.MIS, g, p)
    assert r["best_value"][0] == brute.independence_number(g)
    assert discrete.is_maximal_independent(g, r["best_x"][:, None])[0]


@pytest.mark.parametrize("seed", [0, 1])
def test_solver_finds_brute_force_optimum_maxcut(seed):
    g = graphs.with_weights(graphs.erdos_renyi(16, 0.3, 410 + seed), 420 + seed)
    p = solver.Params(batch=256, steps_per_round=100, rounds=3, alpha=0.05, seed=seed, rho=0.25)
    r = solver.solve(obj.MAXCUT, g, p)
    assert r["best_value"][0] == brute.max_cut(g)
    assert discrete.evaluate_cut(g, r["best_x"][:, None])[0] == r["best_value"][0]


def test_solver_batch_equals_separate_graphs_and_acceptance():
    gs = [graphs.erdos_renyi(30, 0.2, 430), graphs.erdos_renyi(23, 0.3, 431)]
    batch = graphs.concat(gs)
    p = solver.Params(batch=5, steps_per_round=30, rounds=4, alpha=0.02, seed=3)
    r = solver.solve(obj.MIS, batch, p)
    for gi, gg in enumerate(gs):
        vals, zb = solver.solve_graph(obj.MIS, gg, p, graph_index=gi)
        assert np.array_equal(r["traj_best_value"][gi * 5:(gi + 1) * 5], vals)
    # incumbents never decrease and only strict improvements are accepted
    trace = []
    solver.solve_graph(obj.MIS, gs[0], p, 0, trace=trace)
    for a, b in zip(trace, trace[1:]):
        assert np.all(b["best"] >= a["best"])
        assert np.array_equal(b["best"], np.maximum(a["best"], b["value"]))


def test_isolated_vertices_always_in_mis_and_neutral_in_cut():
    g = graphs.concat([graphs.erdos_renyi(20, 0.2, 440), graphs.empty(5)])
    p = solver.Params(batch=4, steps_per_round=50, rounds=2, alpha=0.05, seed=1)
    r = solver.solve(obj.MIS, g, p)
    assert np.all(r["best_x"][20:] == 1)
    assert r["best_value"][1] == 5
    r = solver.solve(obj.MAXCUT, g, p)
    assert r["best_value"][1] == 0


# --------------------------------------------------------------------------
# differentiation: adjoint against central finite differences
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", [obj.MIS, obj.MAXCUT])
def test_unrolled_adjoint_matches_central_differences(kind):
    g = graphs.erdos_renyi(40, 0.1, 501)
    lo, hi = obj.box(kind)
    param = 2.0 if kind == obj.MIS else 1e-3
    K, alpha, h = 6, 0.01, 1e-4
    A = obj.adjacency(g)

    def loss(x0, a):
        xs = pga.unrolled_forward(g, kind, param, a, K, x0)
        return obj.objective(kind, xs[-1], A, param).sum()

    def masks(x0, a):
        out = []
        for xk in pga.unrolled_forward(g, kind, param, a, K, x0)[:-1]:
            z = xk + a * obj.gradient(kind, xk, A, param)
            out.append((z >= lo) & (z <= hi))
        return np.array(out)

    # central differences are valid only where no clip mask changes inside
    # [-h, h]; redraw the start point until that holds (the clipped
    # coordinates themselves are fine: their mask is 0 on both sides)
    for attempt in range(20):
        X0 = arrays.uniform((40, 3), lo, hi, 502 + attempt, np.float64)
        D = arrays.normal(X0.shape, 602 + attempt)
        base = masks(X0, alpha)
        if all(np.array_equal(masks(x, a), base) for x, a in
               ((X0, alpha + h), (X0, alpha - h), (X0 + h * D, alpha), (X0 - h * D, alpha))):
            break
    else:
        pytest.fail("no kink-free start point")
    assert (~base).sum() > 0  # the clip is active somewhere: masks are exercised
    xs = pga.unrolled_forward(g, kind, param, alpha, K, X0)
    dL_dXK = obj.gradient(kind, xs[-1], A, param)
    gx0, galpha = pga.unrolled_backward(g, kind, param, alpha, K, X0, dL_dXK)
    # x_K is a degree-K polynomial in alpha, so the central difference has an
    # O(h^2) term; Richardson extrapolation removes it
    fd_a = (loss(X0, alpha + h) - loss(X0, alpha - h)) / (2 * h)
    fd_a2 = (loss(X0, alpha + h / 2) - loss(X0, alpha - h / 2)) / h
    assert np.isclose(galpha.sum(), fd_a, rtol=1e-4)
    assert np.isclose(galpha.sum(), (4 * fd_a2 - fd_a) / 3, rtol=1e-7)
    fd_x = (loss(X0 + h * D, alpha) - loss(X0 - h * D, alpha)) / (2 * h)
    assert np.isclose((gx0 * D).sum(), fd_x, rtol=1e-6, atol=1e-6)
    # K = 0: the map is the identity
    g0, a0 = pga.unrolled_backward(g, kind, param, alpha, 0, X0, dL_dXK)
    assert np.array_equal(g0, dL_dXK) and np.all(a0 == 0)
