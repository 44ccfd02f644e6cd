"""Pins of the chain's counter-based generator (Algorithm 1 needs a momentum
draw and a Metropolis-Hastings uniform per move).

The integer generator is Philox4x64-10; NumPy ships an independent
implementation of the same generator (numpy.random.Philox), which advances
its counter before each block, so block c of NumPy's stream is the reference
block at counter c + 1.  The uniform and normal transforms are pinned by
their distributions.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import rng


@pytest.mark.parametrize("key,counter", [((1, 2), (0, 0, 0, 0)),
                                         ((0xDEADBEEF12345678, 7), (5, 3, 1, 0)),
                                         ((2 ** 64 - 1, 2 ** 63), (2 ** 64 - 3, 9, 2, 2 ** 64 - 1))])
def test_philox_matches_numpy_bit_generator(key, counter):
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(counter, dtype=np.uint64))
    raw = [int(x) for x in bg.random_raw(12)]
    c = list(counter)
    for b in range(3):
        # NumPy increments the 256-bit counter (word 0 lowest) before a block
        for w in range(4):
            c[w] = (c[w] + 1) % 2 ** 64
            if c[w] != 0:
                break
        assert list(rng.philox4x64(c, key)) == raw[4 * b:4 * b + 4]


def test_uniform53_range_and_resolution():
    assert rng.uniform53(0) == 0.5 * 2.0 ** -53
    assert rng.uniform53(2 ** 64 - 1) == 1.0 - 0.5 * 2.0 ** -53
    assert 0.0 < rng.uniform53(2 ** 11 - 1) == rng.uniform53(0) < rng.uniform53(2 ** 11)


def test_momentum_normals_distribution():
    z = np.concatenate([rng.momentum_normals(11, 3, m, 1001) for m in range(20)])
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / z.size)


def test_streams_moves_and_purposes_are_distinct():
    a = rng.momentum_normals(0, 0, 0, 8)
    assert not np.array_equal(a, rng.momentum_normals(0, 1, 0, 8))     # stream
    assert not np.array_equal(a, rng.momentum_normals(0, 0, 1, 8))     # move
    assert not np.array_equal(a, rng.momentum_normals(1, 0, 0, 8))     # seed
    # a prefix of a longer draw is the shorter draw (blocks are per index)
    assert np.array_equal(rng.momentum_normals(0, 0, 0, 5), a[:5])
    u = [rng.mh_uniform(0, 0, m) for m in range(200)]
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    # the uniform comes from purpose 1, not from the momentum blocks
    w = rng.philox4x64((0, 0, rng.PURPOSE_MOMENTUM, 0), (0, 0))
    assert u[0] != rng.uniform53(w[0])


def test_box_muller_pair():
    r, t = 0.3, 0.2
    z0, z1 = rng.box_muller(r, t)
    assert math.isclose(z0 * z0 + z1 * z1, -2.0 * math.log(r), rel_tol=1e-14)
    assert math.isclose(math.atan2(z1, z0), 2 * math.pi * t, rel_tol=1e-14)
