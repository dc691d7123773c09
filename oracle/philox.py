"""Philox4x64-10 counter-based generator, written from its published
definition (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11): two 64x64->128 multiplications per round with
multipliers 0xD2E7470EE14C6C93 / 0xCA5A826395121157, key bumped by the
Weyl constants 0x9E3779B97F4A7C15 / 0xBB67AE8584CAA73B, ten rounds.

The paper fixes no generator; it only says R is drawn uniformly at random
(Sec. 4) and that x0 is random (Alg. 1 / Alg. 3 initialisation).  Every
random number the method draws comes from this stream:

  key     = (seed, purpose)
  counter = (v >> 3, trajectory, round, 0)
  the 4 output words give 8 uint32 lanes; vertex v takes lane v & 7,
  i.e. word (v & 7) >> 1, low half when v is even, high half when odd.

Test infrastructure only (see ``oracle/__init__``).
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1

PURPOSE_INIT = 1
PURPOSE_RESET = 2
PURPOSE_LS = 3
PURPOSE_NOISE = 4
PURPOSE_SWAP = 5
PURPOSE_POOL = 8


def philox4x64_10(ctr, key):
    """Scalar reference on Python integers: returns the 4 output words."""
    c = [int(x) & MASK64 for x in ctr]
    k0, k1 = int(key[0]) & MASK64, int(key[1]) & MASK64
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k0, p1 & MASK64, (p0 >> 64) ^ c[3] ^ k1, p0 & MASK64]
    return c


_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: int, b: np.ndarray):
    """(hi, lo) of the 128-bit product of the constant ``a`` and uint64 ``b``."""
    a0, a1 = np.uint64(a & 0xFFFFFFFF), np.uint64(a >> 32)
    b0, b1 = b & _M32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _M32) + (p10 & _M32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = (mid << _S32) | (p00 & _M32)
    return hi, lo


def philox4x64_10_np(c0, c1, c2, c3, key0: int, key1: int):
    """Vectorised form over uint64 counter arrays (broadcasting)."""
    with np.errstate(over="ignore"):
        c = list(np.broadcast_arrays(*[np.asarray(x, dtype=np.uint64) for x in (c0, c1, c2, c3)]))
        c = [x.copy() for x in c]
        k0, k1 = key0 & MASK64, key1 & MASK64
        for r in range(10):
            if r:
                k0 = (k0 + W0) & MASK64
                k1 = (k1 + W1) & MASK64
            hi0, lo0 = _mulhilo(M0, c[0])
            hi1, lo1 = _mulhilo(M1, c[2])
            c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
        return c


def vertex_u32(seed: int, purpose: int, traj, rnd: int, v) -> np.ndarray:
    """uint32 draw of vertex ``v`` (local index) for trajectory ``traj`` in
    round ``rnd``; ``traj`` and ``v`` broadcast (e.g. v[:, None], traj[None, :])."""
    v = np.asarray(v, dtype=np.uint64)
    traj = np.asarray(traj, dtype=np.uint64)
    words = philox4x64_10_np(v >> np.uint64(3), traj, np.uint64(rnd), np.uint64(0), seed, purpose)
    lane = v & np.uint64(7)
    w = np.where(lane >> np.uint64(1) == 0, words[0],
                 np.where(lane >> np.uint64(1) == 1, words[1],
                          np.where(lane >> np.uint64(1) == 2, words[2], words[3])))
    shift = (lane & np.uint64(1)) * np.uint64(32)
    return ((w >> shift) & _M32).astype(np.uint32)


def vertex_pair_u32(seed: int, purpose: int, traj, rnd: int, v):
    """Two independent uint32 draws per vertex: both halves of word v & 3 of
    counter (v >> 2, traj, rnd, 0).  Used for the Gaussian noise of the
    degree-based initialisation."""
    v = np.asarray(v, dtype=np.uint64)
    traj = np.asarray(traj, dtype=np.uint64)
    words = philox4x64_10_np(v >> np.uint64(2), traj, np.uint64(rnd), np.uint64(0), seed, purpose)
    j = v & np.uint64(3)
    w = np.where(j == 0, words[0], np.where(j == 1, words[1], np.where(j == 2, words[2], words[3])))
    return (w & _M32).astype(np.uint32), (w >> _S32).astype(np.uint32)


def u32_to_unit_f32(u: np.ndarray) -> np.ndarray:
    """Top 24 bits of a uint32 as an exact float32 in [0, 1)."""
    return ((np.asarray(u, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) * 2.0**-24).astype(np.float32)
