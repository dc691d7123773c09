"""The MaxCut formulations of Sec. 3 besides f_B -- Laplacian f_L (Eq. (4)),
perturbed Laplacian f_P (Eq. (5)), adjacency f_A (Eq. (6)) -- in the CPU
oracle, pinned to the paper's statements about them."""
import itertools

import numpy as np
import pytest

from synth import graphs, arrays
from oracle import objectives as obj, discrete, pga

FORMS = [obj.MAXCUT, obj.MAXCUT_L, obj.MAXCUT_P, obj.MAXCUT_A]


def _spins(n):
    return np.array(list(itertools.product([-1, 1], repeat=n)), dtype=np.float64).T


@pytest.mark.parametrize("kind", FORMS)
@pytest.mark.parametrize("weighted", [False, True])
def test_gradient_central_differences(kind, weighted):
    g = graphs.erdos_renyi(30, 0.2, 800)
    if weighted:
        g = graphs.with_weights(g, 801)
    A = obj.adjacency(g)
    X = arrays.uniform((g.n, 3), -1.0, 1.0, 802).astype(np.float64)
    G = obj.gradient(kind, X, A, 0.3)
    h = 1e-3  # exact for a quadratic up to rounding
    for v in range(0, g.n, 7):
        E = np.zeros_like(X)
        E[v] = h
        fd = (obj.objective(kind, X + E, A, 0.3) - obj.objective(kind, X - E, A, 0.3)) / (2 * h)
        assert np.allclose(fd, G[v], rtol=1e-9, atol=1e-9)
    # the Hessian-vector product is the gradient's linear part
    M = arrays.uniform((g.n, 3), -1.0, 1.0, 803).astype(np.float64)
    assert np.allclose(obj.hessian_vec(kind, A, 0.3, M), G - obj.gradient(kind, X - M, A, 0.3), atol=1e-9)


def test_laplacian_is_the_cut_and_adjacency_differs_by_a_constant():
    """Eq. (4): f_L = Cut on {-1,1}^n; Eq. (6): f_A differs from f_L by a
    constant there (f_A = 4 f_L - sum of weights)."""
    for weighted in (False, True):
        g = graphs.erdos_renyi(8, 0.5, 810)
        if weighted:
            g = graphs.with_weights(g, 811, values=(1, 2, 3))
        A = obj.adjacency(g)
        S = _spins(g.n)
        cut = discrete.evaluate_cut(g, S.astype(np.int8))
        assert np.allclose(obj.f_L(S, A), cut)
        wsum = A.sum()
        assert np.allclose(obj.f_A(S, A), 4 * cut - wsum)


def test_laplacian_stationary_points_have_zero_cut():
    """Prop. 3.2: c 1 is stationary for f_L (a PGA fixed point), interior
    for |c| < 1, binary for c = +-1, and its cut is 0."""
    g = graphs.erdos_renyi(40, 0.3, 820)
    A = obj.adjacency(g)
    for c in (-1.0, -0.375, 0.0, 0.5, 1.0):  # dyadic: the row sums are exact
        X = np.full((g.n, 1), c)
        assert np.allclose(obj.grad_f_L(X, A), 0.0)
        Y, _ = pga.step64(X, A, obj.MAXCUT_L, 0.1, 0.0)
        assert np.array_equal(Y, X)
    assert discrete.evaluate_cut(g, discrete.round_x(obj.MAXCUT_L, np.full((g.n, 1), 0.5)))[0] == 0


def test_perturbed_laplacian_fixes_every_binary_point():
    """Thm. 3.3: for lambda > 0 every x in {-1,1}^n is a PGA fixed point of f_P."""
    g = graphs.erdos_renyi(9, 0.45, 830)
    A = obj.adjacency(g)
    S = _spins(g.n)
    for lam, alpha in ((1e-3, 0.1), (0.5, 0.01)):
        Y, _ = pga.step64(S, A, obj.MAXCUT_P, alpha, lam)
        assert np.array_equal(Y, S)


def test_adjacency_escapes_one_flip_repairable_points():
    """Prop. 3.4: a binary x that one flip improves is not a PGA fixed point
    of f_A."""
    g = graphs.erdos_renyi(9, 0.45, 840)
    A = obj.adjacency(g)
    S = _spins(g.n)
    repairable = np.any(discrete.gains(obj.MAXCUT, g, S.astype(np.int8)) > 0, axis=0)
    Y, _ = pga.step64(S, A, obj.MAXCUT_A, 0.1, 0.0)
    moved = np.any(Y != S, axis=0)
    assert repairable.any()
    assert np.all(moved[repairable])


@pytest.mark.parametrize("kind", FORMS)
def test_float32_replay_close_to_float64(kind):
    g = graphs.with_weights(graphs.erdos_renyi(60, 0.1, 850), 851)
    X = arrays.uniform((g.n, 4), -1.0, 1.0, 852)
    y32, _ = pga.step32(g, X, kind, 0.05, 0.2)
    y64, _ = pga.step64(X.astype(np.float64), obj.adjacency(g), kind, 0.05, 0.2)
    assert np.abs(y32 - y64).max() <= 1e-5


def _run_to_convergence(kind, A, X, alpha, steps):
    for _ in range(steps):
        Y, _ = pga.step64(X, A, kind, alpha, 1e-3)
        if np.array_equal(Y, X):
            break
        X = Y
    return X


def test_escape_from_c1_cut_at_convergence():
    """App. B's first escapability set-up (ER(100, 0.66), x0 = c 1,
    lambda = 1e-3), with the cut recorded at convergence in float64.
    Exact arithmetic: c 1 is stationary for f_L (Prop. 3.2) and PGA on f_P
    stays uniform (its gradient there is 2 lambda c 1), so both end at cut 0;
    f_B's gradient -lambda - 2 c d varies with the degree d.  Float64: the
    row sums of L (c 1) are exactly zero only when c d is exact (c = 0.375);
    otherwise their rounding grows by the ascent on the positive
    semi-definite x^T L x and f_L and f_P leave the diagonal to large cuts.
    f_B at the appendix's alpha = 0.1 overshoots: within two steps every
    coordinate sits at the same bound, and the iterate alternates between
    -1 and +1 with cut 0; at alpha = 1e-3 it converges to cuts near 1800."""
    g = graphs.erdos_renyi(100, 0.66, 700)
    A = obj.adjacency(g)
    cs = np.array([[-0.83, -0.07, 0.3, 0.77]])
    X0 = np.repeat(cs, g.n, 0)
    cut = lambda kind, X: discrete.evaluate_cut(g, discrete.round_x(kind, X))  # noqa: E731
    # f_L from an exactly representable c 1: stationary, nothing moves
    X = np.full((g.n, 1), 0.375)
    assert np.array_equal(_run_to_convergence(obj.MAXCUT_L, A, X, 0.1, 50), X)
    assert cut(obj.MAXCUT_L, X)[0] == 0
    # f_P from an exact c 1: the exact gradient is 2 lambda c 1
    assert np.array_equal(obj.grad_f_P(X, A, 1e-3), np.full((g.n, 1), 2 * 1e-3 * 0.375))
    # float64 rounding: f_L and f_P escape from generic c (f_P also from 0.375)
    assert np.all(cut(obj.MAXCUT_L, _run_to_convergence(obj.MAXCUT_L, A, X0, 0.1, 200)) >= 1300)
    XP = np.concatenate([X0, X], 1)
    assert np.all(cut(obj.MAXCUT_P, _run_to_convergence(obj.MAXCUT_P, A, XP, 0.1, 200)) >= 1300)
    # f_B at alpha = 0.1: a uniform +-1 iterate after two steps, cut 0
    XB = X0
    for _ in range(2):
        XB, _ = pga.step64(XB, A, obj.MAXCUT, 0.1, 1e-3)
    assert np.all(np.abs(XB) == 1) and np.all(XB == XB[:1])
    XB2, _ = pga.step64(XB, A, obj.MAXCUT, 0.1, 1e-3)
    assert np.array_equal(XB2, -XB) and np.all(cut(obj.MAXCUT, XB) == 0)
    # f_B at alpha = 1e-3 leaves the diagonal in exact arithmetic too
    assert np.all(cut(obj.MAXCUT, _run_to_convergence(obj.MAXCUT, A, X0, 1e-3, 1500)) >= 1750)
