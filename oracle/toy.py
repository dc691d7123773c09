"""Prop. 4.1's separable toy: the unbiased single-coordinate global reset
against full random restarts (Sec. 4, proof in the appendix).

Minimise F(x) = sum_i phi(x_i) over [-1,1]^n with the double well
    phi(x) = -x^2/2 - beta x^3 / 3,  0 < beta < 1,
whose only stationary point inside the box is x = 0 (phi'(x) = -x (1 + beta
x)); projected gradient descent x <- Pi(x + alpha (x + beta x^2)) sends a
start in (0, 1] to 1 and a start in [-1, 0) to -1, and phi(1) < phi(-1), so
x* = (1, ..., 1).  (The proposition fixes only these properties; this phi
is one function that has them.)

Random numbers: Philox4x64-10 (``philox``) with purpose TOY_RESET for the
reset attempts and TOY_START for the restart draws.  A value draw w (uint32)
gives y = (2 (w >> 8) + 1 - 2^24) / 2^24, an exact float32 that is never 0,
symmetric about 0.  Attempt a of trial t draws the coordinate i =
(w0 * n) >> 32 from lane 0 and the value from lane 1 of counter
(0, t, a, 0); restart j of trial t draws coordinate v's value from lane v of
counter (v >> 3, t, j, 0).

* Global reset (the proposition's mQO variant): start from restart 0's
  descended point; every attempt resets one coordinate to y, descends it for
  ``steps`` float32 steps, and keeps it iff phi strictly decreases.
* Full restart: restarts j = 1, 2, ... descend a fresh point from the
  draws; success when it is x*.

Each trial reports the first attempt (restart) index after which the point
is x*, or -1.  Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from . import philox

PURPOSE_TOY_RESET = 6
PURPOSE_TOY_START = 7
F32 = np.float32


def phi(x, beta):
    """float64, in the order written: a = x x, b = a x, -0.5 a - (beta b) / 3."""
    x = np.asarray(x, dtype=np.float64)
    a = x * x
    b = a * x
    return -0.5 * a - (beta * b) / 3.0


def value_from_u32(w):
    k = (np.asarray(w, dtype=np.uint32) >> np.uint32(8)).astype(np.int64)
    return ((2 * k + 1 - (1 << 24)).astype(F32) * F32(2.0 ** -24)).astype(F32)


def descend32(y, alpha, beta, steps):
    """``steps`` projected descent steps on phi, float32, one rounding per
    operation: t = y*y, t = beta*t, t = y + t, t = alpha*t, y = y + t, clip."""
    y = np.array(y, dtype=F32)
    a, b = F32(alpha), F32(beta)
    for _ in range(steps):
        t = y * y
        t = b * t
        t = y + t
        t = a * t
        y = np.minimum(np.maximum(y + t, F32(-1.0)), F32(1.0))
    return y


def start_points(seed, n, trials, j, alpha, beta, steps):
    """Descended restart j of every trial: float32 [trials][n]."""
    t = np.arange(trials, dtype=np.uint64)[:, None]
    v = np.arange(n, dtype=np.uint64)[None, :]
    w = philox.vertex_u32(seed, PURPOSE_TOY_START, t, j, v)
    return descend32(value_from_u32(w), alpha, beta, steps)


def global_reset(seed, n, trials, attempts, alpha=0.5, beta=0.5, steps=128):
    """Returns (first_hit int64[trials], final point float32[trials][n])."""
    x = start_points(seed, n, trials, 0, alpha, beta, steps)
    t = np.arange(trials, dtype=np.uint64)
    first = np.where(np.all(x == F32(1.0), axis=1), 0, -1).astype(np.int64)
    rows = np.arange(trials)
    for a in range(attempts):
        w0 = philox.vertex_u32(seed, PURPOSE_TOY_RESET, t, a, np.uint64(0))
        w1 = philox.vertex_u32(seed, PURPOSE_TOY_RESET, t, a, np.uint64(1))
        i = ((w0.astype(np.uint64) * np.uint64(n)) >> np.uint64(32)).astype(np.int64)
        y = descend32(value_from_u32(w1), alpha, beta, steps)
        old = x[rows, i]
        take = phi(y, beta) < phi(old, beta)
        x[rows[take], i[take]] = y[take]
        hit = (first < 0) & np.all(x == F32(1.0), axis=1)
        first[hit] = a + 1
    return first, x


def full_restart(seed, n, trials, restarts, alpha=0.5, beta=0.5, steps=128):
    """First restart index j >= 1 whose descended point is x* (-1 if none
    within ``restarts``), and whether restart 0 already was."""
    first = np.full(trials, -1, dtype=np.int64)
    start_hit = np.all(start_points(seed, n, trials, 0, alpha, beta, steps) == F32(1.0), axis=1)
    for j in range(1, restarts + 1):
        hit = (first < 0) & np.all(start_points(seed, n, trials, j, alpha, beta, steps) == F32(1.0), axis=1)
        first[hit] = j
    return np.where(start_hit, 0, first), start_hit


def success_probability(n, k0, m):
    """Exact P(x* after m attempts | k0 coordinates start at -1): every
    attempt corrects a given wrong coordinate with probability 1/(2n) and
    never two at once, so by inclusion-exclusion
    sum_j (-1)^j C(k0, j) (1 - j/(2n))^m."""
    from math import comb
    return sum((-1) ** j * comb(k0, j) * (1.0 - j / (2.0 * n)) ** m for j in range(k0 + 1))


def failure_bound(n, rounds):
    """The proposition's union bound after ``rounds`` rounds of n attempts:
    n exp(-rounds / 2)."""
    return n * np.exp(-rounds / 2.0)
