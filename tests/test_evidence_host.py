"""The evidence pipeline's host arithmetic against the reference: the same
rung schedule, and the same trapezoid estimate and variance on shared
values (no GPU)."""
import numpy as np

from oracle import evidence as oev
from paper_2511_06407_amd import evidence as ev


def test_schedule_matches_reference():
    assert np.array_equal(ev.paper_schedule().round(15), oev.paper_schedule().round(15))


def test_trapezoid_matches_reference():
    rng = np.random.default_rng(0)
    t = oev.paper_schedule()
    L = rng.standard_normal((7, t.size)) * 2.0 - 40.0 * t
    est, var, E = ev.trapezoid(t, L)
    rest, rvar, rE = oev.ti_estimate(t, L)
    assert abs(est - rest) < 1e-12 * abs(rest)
    assert abs(var - rvar / 7) < 1e-12 * rvar
    assert np.allclose(E, rE, rtol=0, atol=0)
