"""Counter-based random numbers of the chain: Philox4x64-10 and Box-Muller.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 1 draws a momentum p ~ N(0, G(q)) at the start of every move and
one uniform r for the Metropolis-Hastings test.  So that the FP64 reference
and the device chain consume identical randomness without exchanging arrays,
both derive it from one counter-based generator, each side implementing it
on its own from the published definition:

* Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC 2011): a 4 x 64-bit counter and a 2 x 64-bit key; ten
  rounds, each multiplying counter words 0 and 2 by two fixed odd constants
  into 128-bit products, mixing the high halves with the other two counter
  words and the key, and bumping the key by two Weyl constants between
  rounds.
* key = (seed, stream_id); counter = (block j, move l, purpose, 0) with
  purpose 0 for the momentum normals of move l and 1 for its uniform.
* A 64-bit word w becomes u = ((w >> 11) + 1/2) 2^-53, strictly inside (0, 1).
* Normals by the Box-Muller transform: a pair of uniforms (u0, u1) gives
  sqrt(-2 ln u0) cos(2 pi u1) and sqrt(-2 ln u0) sin(2 pi u1); block j yields
  normals 4j .. 4j+3 from its words (0, 1) and (2, 3).
* The Metropolis-Hastings uniform of move l is word 0 of block 0 of purpose 1.

Only the integer generator is pinned bit for bit (against NumPy's own
Philox bit generator); the two sides' log, sqrt, sin and cos may differ in
the last place, which moves a normal by an ulp.
"""
from __future__ import annotations

import math

import numpy as np

_MASK = (1 << 64) - 1
PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)   # round multipliers
PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)   # key increments (Weyl)
PHILOX_ROUNDS = 10

PURPOSE_MOMENTUM = 0
PURPOSE_UNIFORM = 1


def philox4x64(counter, key, rounds=PHILOX_ROUNDS):
    """One Philox4x64 block: four 64-bit output words for a 4-word counter and
    a 2-word key (Python ints)."""
    c0, c1, c2, c3 = (int(x) & _MASK for x in counter)
    k0, k1 = (int(x) & _MASK for x in key)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + PHILOX_W[0]) & _MASK
            k1 = (k1 + PHILOX_W[1]) & _MASK
        p0 = PHILOX_M[0] * c0
        p1 = PHILOX_M[1] * c2
        hi0, lo0 = p0 >> 64, p0 & _MASK
        hi1, lo1 = p1 >> 64, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniform53(w):
    """(0, 1) uniform from the top 53 bits of a 64-bit word."""
    return ((int(w) >> 11) + 0.5) * (2.0 ** -53)


def box_muller(u0, u1):
    r = math.sqrt(-2.0 * math.log(u0))
    t = 2.0 * math.pi * u1
    return r * math.cos(t), r * math.sin(t)


def momentum_normals(seed, stream_id, move, D):
    """The D standard normals z of move `move` (p = G^{1/2} z)."""
    z = np.empty(D)
    for j in range((D + 3) // 4):
        w = philox4x64((j, move, PURPOSE_MOMENTUM, 0), (seed, stream_id))
        a = box_muller(uniform53(w[0]), uniform53(w[1]))
        b = box_muller(uniform53(w[2]), uniform53(w[3]))
        for k, v in enumerate(a + b):
            i = 4 * j + k
            if i < D:
                z[i] = v
    return z


def mh_uniform(seed, stream_id, move):
    """The Metropolis-Hastings uniform r of move `move`."""
    w = philox4x64((0, move, PURPOSE_UNIFORM, 0), (seed, stream_id))
    return uniform53(w[0])


def chain_randoms(seed, stream_id, n_moves, D):
    """(z, u): n_moves x D normals and n_moves uniforms of a seeded chain."""
    z = np.stack([momentum_normals(seed, stream_id, m, D) for m in range(n_moves)]) \
        if n_moves else np.empty((0, D))
    u = np.array([mh_uniform(seed, stream_id, m) for m in range(n_moves)])
    return z, u
