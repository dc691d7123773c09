"""Pins of the CPU oracle against what the paper and the mathematics fix:
closed forms, theorem statements, worked examples, brute force and
library routines.  CPU only."""
import json
import os

import numpy as np
import pytest

from synth import graphs, arrays
from oracle import philox, objectives as obj, pga, discrete, brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dense(g):
    A = np.zeros((g.n, g.n))
    u, v, w = g.edges()
    A[u, v] = w
    A[v, u] = w
    return A


# --------------------------------------------------------------------------
# Philox: the oracle's generator equals numpy's independent implementation
# --------------------------------------------------------------------------

@pytest.mark.parametrize("ctr,key", [((0, 0, 0, 0), (0, 0)), ((1, 2, 3, 4), (5, 6)),
                                     ((2**64 - 1, 7, 9, 11), (123456789, 987654321)),
                                     ((12345, 678, 9, 3), (2**63 + 5, 2))])
def test_philox_matches_numpy(ctr, key):
    # numpy's Philox bumps the counter before generating its first block
    whole = sum(c << (64 * i) for i, c in enumerate(ctr))
    whole = (whole - 1) % 2**256
    prev = [(whole >> (64 * i)) & (2**64 - 1) for i in range(4)]
    bg = np.random.Philox(counter=np.array(prev, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    ref = [int(x) for x in bg.random_raw(4)]
    assert philox.philox4x64_10(ctr, key) == ref
    vec = philox.philox4x64_10_np(*[np.uint64(c) for c in ctr], key[0], key[1])
    assert [int(x) for x in vec] == ref


def test_vertex_lane_layout():
    v = np.arange(40, dtype=np.uint64)
    got = philox.vertex_u32(77, philox.PURPOSE_RESET, 5, 3, v)
    for vi in range(40):
        w = philox.philox4x64_10((vi >> 3, 5, 3, 0), (77, philox.PURPOSE_RESET))
        lane = vi & 7
        exp = (w[lane >> 1] >> (32 * (lane & 1))) & 0xFFFFFFFF
        assert int(got[vi]) == exp
    u = philox.u32_to_unit_f32(got)
    assert u.dtype == np.float32 and np.all(u >= 0) and np.all(u < 1)
    assert np.all(u.astype(np.float64) * 2**24 == np.floor(u.astype(np.float64) * 2**24))


# --------------------------------------------------------------------------
# objectives against their edge-sum definitions and finite differences
# --------------------------------------------------------------------------

def _fd_grad(f, X, h=1e-4):
    G = np.zeros_like(X)
    for v in range(X.shape[0]):
        E = np.zeros_like(X)
        E[v] = h
        G[v] = (f(X + E) - f(X - E)) / (2 * h)
    return G


@pytest.mark.parametrize("weighted", [False, True])
def test_objectives_edge_forms_and_fd(weighted):
    g = graphs.erdos_renyi(30, 0.2, 11)
    if weighted:
        g = graphs.with_weights(g, 12, values=(-2, -1, 1, 3))
    A = obj.adjacency(g)
    u, v, w = g.edges()
    X = arrays.uniform((30, 4), -1, 1, 13, np.float64)
    gamma, lam = 2.5, 0.3
    # Eq. (3) first form: sum_v x_v - gamma sum_(u,v) in E x_u x_v  (unit weights only)
    if not weighted:
        h_edges = X.sum(0) - gamma * (X[u] * X[v]).sum(0)
        assert np.allclose(obj.h(X, A, gamma), h_edges, rtol=0, atol=1e-12)
    # Eq. (7): -lambda 1^T x - x^T A x, with x^T A x = 2 sum_E w x_u x_v
    fb_edges = -lam * X.sum(0) - 2 * (w[:, None] * X[u] * X[v]).sum(0)
    assert np.allclose(obj.f_B(X, A, lam), fb_edges, rtol=0, atol=1e-12)
    # central differences are exact up to rounding for quadratics
    assert np.allclose(obj.grad_f_B(X, A, lam), _fd_grad(lambda Y: obj.f_B(Y, A, lam), X), atol=1e-7)
    assert np.allclose(obj.grad_h(X, A, gamma), _fd_grad(lambda Y: obj.h(Y, A, gamma), X), atol=1e-7)


def test_laplacian_cut_identity_and_gain_identity():
    g = graphs.with_weights(graphs.erdos_renyi(25, 0.3, 21), 22)
    A = obj.adjacency(g)
    S = arrays.spins((25, 6), 23)
    cut = discrete.evaluate_cut(g, S)
    # Eq. (4): on {-1,1}^n, f_L = (1/4) x^T L x = Cut(S)
    assert np.allclose(obj.f_L(S.astype(np.float64), A), cut)
    # 1-flip gain (proof of Prop. 3.4): Cut(x^(i)) - Cut(x) = x_i (A x)_i, for every i
    gains = discrete.gains(obj.MAXCUT, g, S)
    for i in range(25):
        S2 = S.copy()
        S2[i] *= -1
        assert np.array_equal(discrete.evaluate_cut(g, S2) - cut, gains[i])
    # the same identity through f_A: f_A(x^(i)) - f_A(x) = 4 x_i (A x)_i
    fa = obj.f_A(S.astype(np.float64), A)
    S2 = S.copy()
    S2[3] *= -1
    assert np.allclose(obj.f_A(S2.astype(np.float64), A) - fa, 4 * gains[3])


def test_mis_gains_match_h_differences():
    g = graphs.erdos_renyi(20, 0.25, 31)
    A = obj.adjacency(g)
    Z = arrays.binary01((20, 5), 32)
    gamma = 2.0
    base = obj.h(Z.astype(np.float64), A, gamma)
    gains = discrete.gains(obj.MIS, g, Z, gamma)
    for v in range(20):
        Z2 = Z.copy()
        Z2[v] = 1 - Z2[v]
        assert np.allclose(obj.h(Z2.astype(np.float64), A, gamma) - base, gains[v])


# --------------------------------------------------------------------------
# theorem statements and worked examples
# --------------------------------------------------------------------------

def test_prop31_p3_swap_repairable_point_is_fixed():
    ex = json.load(open(os.path.join(GOLDEN, "p3_swap_example.json")))
    g = graphs.from_edges(ex["n"], [e[0] for e in ex["edges"]], [e[1] for e in ex["edges"]])
    A = obj.adjacency(g)
    x = np.array(ex["x"], dtype=np.float64)[:, None]
    sw = np.array(ex["swap_result"])[:, None]
    # the swap result is independent and one larger (Def. 2.3)
    size, conf = discrete.evaluate_mis(g, sw)
    assert conf[0] == 0 and size[0] == x.sum() + 1
    for gamma in ex["gammas"]:
        for alpha in ex["alphas"]:
            x1, _ = pga.step64(x, A, obj.MIS, alpha, gamma)
            assert np.array_equal(x1, x)


def test_prop32_constant_vectors_stationary_for_fL():
    g = graphs.erdos_renyi(15, 0.4, 41)
    A = obj.adjacency(g)
    for c in (-0.7, 0.0, 0.3, 1.0):
        X = np.full((15, 1), c)
        assert np.allclose(_fd_grad(lambda Y: obj.f_L(Y, A), X), 0, atol=1e-9)


def test_thm33_every_binary_point_fixed_for_fP():
    g = graphs.erdos_renyi(12, 0.4, 51)
    A = obj.adjacency(g)
    lam = 0.01
    S = arrays.spins((12, 20), 52).astype(np.float64)
    grad = _fd_grad(lambda Y: obj.f_P(Y, A, lam), S)
    for alpha in (0.01, 0.3):
        assert np.array_equal(np.clip(S + alpha * grad, -1, 1), S)


def test_thm36_i_repairable_points_move_under_fB():
    g = graphs.erdos_renyi(40, 0.2, 61)
    A = obj.adjacency(g)
    S = arrays.spins((40, 64), 62)
    gains = discrete.gains(obj.MAXCUT, g, S)
    rep = np.any(gains > 0, axis=0)
    assert rep.sum() > 10
    for lam in (1e-3, 0.5, 1.99):
        X1, _ = pga.step64(S.astype(np.float64), A, obj.MAXCUT, 0.05, lam)
        moved = X1 != S
        # every 1-flip repairable coordinate moves, so every repairable point moves
        assert np.all(moved[gains > 0])
        assert np.all(np.any(moved, axis=0)[rep])
    # the bound lambda < 2 is sharp: on the 2-path at s = (-1, -1) both flips
    # gain 1, x_i grad_i = lambda - 2, so lambda = 2 stalls and lambda < 2 moves
    g2 = graphs.path(2)
    s = np.array([[-1.0], [-1.0]])
    assert np.all(discrete.gains(obj.MAXCUT, g2, s.astype(np.int8)) == 1)
    X1, _ = pga.step64(s, obj.adjacency(g2), obj.MAXCUT, 0.05, 2.0)
    assert np.array_equal(X1, s)
    X1, _ = pga.step64(s, obj.adjacency(g2), obj.MAXCUT, 0.05, 1.99)
    assert np.all(X1 > -1.0)
    # a point without positive gains (the edge is cut) is fixed
    s = np.array([[1.0], [-1.0]])
    X1, _ = pga.step64(s, obj.adjacency(g2), obj.MAXCUT, 0.05, 1e-3)
    assert np.array_equal(X1, s)


def test_thm36_ii_limits_are_binary():
    for seed in range(3):
        g = graphs.erdos_renyi(30, 0.2, 70 + seed)
        A = obj.adjacency(g)
        X = arrays.uniform((30, 16), -1, 1, 80 + seed, np.float64)
        # lambda = 0.5 so that balanced coordinates (gradient -lambda) do
        # not take tens of thousands of steps to reach the boundary
        for _ in range(3000):
            X, _ = pga.step64(X, A, obj.MAXCUT, 0.05, 0.5)
        X1, _ = pga.step64(X, A, obj.MAXCUT, 0.05, 0.5)
        assert np.array_equal(X1, X)  # a PGA fixed point
        iso = np.diff(g.row_ptr) == 0
        # isolated vertices: gradient -lambda drives them to -1 as well
        assert np.all(np.abs(X[~iso]) == 1.0)
        assert np.all(X[iso] == -1.0)


def test_k3_adjacency_example():
    ex = json.load(open(os.path.join(GOLDEN, "k3_adjacency_example.json")))
    g = graphs.from_edges(ex["n"], [e[0] for e in ex["edges"]], [e[1] for e in ex["edges"]])
    A = obj.adjacency(g)
    s = np.array(ex["binary_maximizer"], dtype=np.float64)
    fa_s = obj.f_A(s[:, None], A)[0]
    allS = 2.0 * brute.all_binary(3).astype(np.float64).T - 1.0
    assert fa_s == obj.f_A(allS, A).max()
    i = ex["balanced_vertex"]
    for t in ex["t_values"]:
        x = s.copy()
        x[i] = t
        assert np.isclose(obj.f_A(x[:, None], A)[0], fa_s)
        # under f_B the balanced coordinate has gradient -lambda != 0
        lam = 1e-3
        assert np.isclose(obj.grad_f_B(x[:, None], A, lam)[i, 0], -lam)


# --------------------------------------------------------------------------
# checker (8) by brute force
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_checker_fixed_points_are_maximal_independent_sets(seed):
    n = 11
    g = graphs.erdos_renyi(n, 0.3, 90 + seed)
    mis_sets = brute.maximal_independent_sets(g)
    Z = brute.all_binary(n).T  # [n][2^n]
    for gamma in (1.01, 2.0, 3.0):
        for alpha in (0.01, 1.0):
            fixed = discrete.is_pga_fixed_mis(g, Z, gamma, alpha)
            got = {tuple(int(x) for x in Z[:, j]) for j in np.flatnonzero(fixed)}
            assert got == mis_sets
    assert np.array_equal(discrete.is_maximal_independent(g, Z),
                          discrete.is_pga_fixed_mis(g, Z, 2.0, 0.5))


def test_rounding_is_strict():
    assert discrete.round_mis(np.array([0.5, 0.50001, 0.0, 1.0], dtype=np.float32)).tolist() == [0, 1, 0, 1]
    assert discrete.round_cut(np.array([0.0, -0.0, 1e-30, -1.0], dtype=np.float32)).tolist() == [-1, -1, 1, -1]


def test_evaluate_mis_against_edges():
    g = graphs.erdos_renyi(40, 0.15, 101)
    Z = arrays.binary01((40, 7), 102)
    size, conf = discrete.evaluate_mis(g, Z)
    u, v, _ = g.edges()
    assert np.array_equal(conf, ((Z[u] == 1) & (Z[v] == 1)).sum(0))
    assert np.array_equal(size, Z.sum(0))


@pytest.mark.parametrize("which", ["er", "torus_pm1", "star", "batch"])
def test_float32_neighbour_sums_follow_csr_order(which):
    """The library route of the float32 neighbour sums equals the
    position-by-position definition bit for bit, on values whose sums depend
    on the order of addition (a reversed order changes some of them)."""
    from oracle import pga
    g = {"er": graphs.erdos_renyi(800, 0.03, 61), "torus_pm1": graphs.torus_pm1(40, 62),
         "star": graphs.star(500),
         "batch": graphs.concat([graphs.erdos_renyi(97, 0.08, 63), graphs.empty(3), graphs.star(40)])}[which]
    rng = np.random.default_rng(64)
    X = (rng.uniform(-1, 1, (g.n, 6)) * 10.0 ** rng.integers(-6, 4, (g.n, 6))).astype(np.float32)
    a = pga.neighbour_sum32(g, X)
    assert a.dtype == np.float32
    assert np.array_equal(a, pga.neighbour_sum32_positions(g, X))
    # the order matters on these values: summing each row backwards differs somewhere
    rev = np.zeros_like(X)
    for v in range(g.n):
        for j in range(g.row_ptr[v + 1] - 1, g.row_ptr[v] - 1, -1):
            w = np.float32(1.0) if g.weight is None else np.float32(g.weight[j])
            rev[v] = rev[v] + w * X[g.col_idx[j]]
    assert not np.array_equal(rev, a)
