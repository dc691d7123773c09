"""Pins of the Prop. 4.1 toy oracle: the double well's basins, the exact
success law of the single-coordinate reset, the restart law, and the
proposition's bound.  CPU only."""
from math import log

import numpy as np

from oracle import toy


def _z(obs, p):
    p = np.asarray(p, dtype=np.float64)
    return abs(obs - p.sum()) / np.sqrt(max((p * (1 - p)).sum(), 1e-12))


def test_double_well_shape():
    beta = 0.5
    assert toy.phi(1.0, beta) < toy.phi(-1.0, beta)
    # phi'(x) = -x (1 + beta x): the only zero in [-1, 1] is 0, a maximum
    xs = np.linspace(-1, 1, 2001)
    d = -xs * (1 + beta * xs)
    assert np.all(np.sign(d[xs > 0]) < 0) and np.all(np.sign(d[xs < 0]) > 0)


def test_descent_basins_on_every_slow_draw():
    """Every draw descends to the sign of its value; the draws nearest 0
    (the slowest) are checked exhaustively, the rest on a stride."""
    k = np.concatenate([np.arange((1 << 23) - (1 << 16), (1 << 23) + (1 << 16)),
                        np.arange(0, 1 << 24, 97), [0, (1 << 24) - 1]]).astype(np.uint32)
    y = toy.value_from_u32(k << np.uint32(8))
    assert np.all(y != 0) and y.min() > -1 and y.max() < 1
    d = toy.descend32(y, 0.5, 0.5, 128)
    assert np.array_equal(d, np.where(y > 0, np.float32(1), np.float32(-1)))


def test_value_draws_symmetric():
    """k and 2^24 - 1 - k give opposite values: the reset law is symmetric
    about the basin boundary 0."""
    k = np.arange(0, 1 << 24, 4093, dtype=np.uint32)
    y = toy.value_from_u32(k << np.uint32(8))
    y2 = toy.value_from_u32((np.uint32((1 << 24) - 1) - k) << np.uint32(8))
    assert np.array_equal(y, -y2)


def test_reset_changes_one_coordinate_and_never_worsens():
    n, T = 12, 300
    prev = None
    for a in range(0, 40, 3):
        _, x = toy.global_reset(21, n, T, a)
        if prev is not None:
            f_prev = toy.phi(prev, 0.5).sum(axis=1)
            f = toy.phi(x, 0.5).sum(axis=1)
            assert np.all(f <= f_prev + 1e-12)
            assert np.all((x != prev).sum(axis=1) <= 3)  # three attempts, one coordinate each
        prev = x


def test_global_reset_matches_the_exact_success_law():
    n, T, m = 32, 2000, 400
    first, _ = toy.global_reset(5, n, T, m)
    k0 = (toy.start_points(5, n, T, 0, 0.5, 0.5, 128) < 0).sum(axis=1)
    p = np.array([toy.success_probability(n, int(k), m) for k in k0])
    assert _z((first >= 0).sum(), p) < 4.0
    # and at an intermediate budget
    p2 = np.array([toy.success_probability(n, int(k), m // 4) for k in k0])
    assert _z(((first >= 0) & (first <= m // 4)).sum(), p2) < 4.0


def test_full_restart_matches_its_law():
    n, T, J = 5, 4000, 64
    first, start_hit = toy.full_restart(9, n, T, J)
    q = 2.0 ** -n
    assert _z(start_hit.sum(), np.full(T, q)) < 4.0
    later = ~start_hit
    p = np.full(later.sum(), 1 - (1 - q) ** J)
    assert _z((first[later] > 0).sum(), p) < 4.0


def test_proposition_bound_holds():
    """R >= 2 log(n / delta) rounds of n attempts fail with probability at
    most delta."""
    n, T, delta = 16, 3000, 0.05
    R = int(np.ceil(2 * log(n / delta)))
    first, _ = toy.global_reset(13, n, T, R * n)
    fail = (first < 0).mean()
    assert toy.failure_bound(n, R) <= delta
    assert fail <= delta + 4 * np.sqrt(delta * (1 - delta) / T)
