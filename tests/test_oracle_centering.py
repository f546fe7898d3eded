"""Pins of Algorithm 1 (Section 3.1) in the oracle: hand-computed cases and
invariants implied by the algorithm's definition."""
import numpy as np
import pytest

from oracle.centering import center, reclamp

MU, DELTA, ALPHA = 1e-6, 1e-4, 1e-6  # the parameters Section 3.1 settles on


def test_hand_case_zero_primal():
    # x = 0, z = 0.5 (complementarity 0 -> mu_target = mu_min):
    # x' = max(0, 1e-6) = 1e-6 < z' = 0.5, so x' = clamp(1e-6 / 0.5) = 2e-6,
    # then z' = clamp(1e-6 / 2e-6 = 0.5, 0.5 +- 1e-4) = 0.5
    xp, zp, mu = center([0.0], [0.5], MU, DELTA, ALPHA)
    assert mu == MU
    assert xp[0] == pytest.approx(2e-6, rel=1e-15)
    assert zp[0] == pytest.approx(0.5, rel=1e-15)


def test_hand_case_zero_dual():
    # x = 0.3, z = 0: z' = 1e-6 <= x', so z' moves first: mu / 0.3 = 3.333e-6
    # (inside 1e-6 +- 1e-4); then x' = mu / z' = 0.3 exactly up to rounding
    xp, zp, _ = center([0.3], [0.0], MU, DELTA, ALPHA)
    assert zp[0] == pytest.approx(1e-6 / 0.3, rel=1e-15)
    assert xp[0] == pytest.approx(0.3, rel=1e-15)


def test_hand_case_delta_binds():
    # x = (0.01, 0), z = (0.02, 0): mu_target = (0.01 * 0.02) / 2 = 1e-4.
    # Pair 0: x' = 0.01 < z' = 0.02; x' wants 1e-4 / 0.02 = 5e-3 but may move
    # only 1e-4, so x' = 0.0099; z' wants 1e-4 / 0.0099 = 0.0101 but is held at
    # 0.02 - 1e-4 = 0.0199.
    xp, zp, mu = center([0.01, 0.0], [0.02, 0.0], MU, DELTA, ALPHA)
    assert mu == pytest.approx(1e-4, rel=1e-15)
    assert xp[0] == pytest.approx(0.0099, rel=1e-14)
    assert zp[0] == pytest.approx(0.0199, rel=1e-14)
    # pair 1: both lifted to 1e-6; tie, so z' first: wants 1e-4/1e-6 = 100,
    # held at 1e-6 + 1e-4; then x' wants 1e-4 / 1.01e-4, held at 1.01e-4
    assert zp[1] == pytest.approx(1.01e-4, rel=1e-14)
    assert xp[1] == pytest.approx(1.01e-4, rel=1e-14)


def test_tie_takes_the_else_branch():
    # x' == z': z' is updated first
    xp, zp, mu = center([0.5, 0.0], [0.5, 0.0], MU, DELTA, ALPHA)
    # mu = 0.125: z' = clamp(0.25, 0.5 +- 1e-4) = 0.4999, then
    # x' = clamp(0.125 / 0.4999 = 0.25005, 0.5 +- 1e-4) = 0.4999
    assert zp[0] == pytest.approx(0.5 - DELTA, rel=1e-15)
    assert xp[0] == pytest.approx(0.5 - DELTA, rel=1e-15)


def test_invariants_random():
    rng = np.random.default_rng(4)
    n = 5000
    x = np.where(rng.random(n) < 0.5, 0.0, rng.exponential(1.0, n))
    z = np.where(x > 0, rng.exponential(1e-3, n) * (rng.random(n) < 0.1), rng.exponential(1.0, n))
    xp, zp, mu = center(x, z, MU, DELTA, ALPHA)
    assert mu == max(float(x @ z) / n, MU)
    xl, zl = np.maximum(x, ALPHA), np.maximum(z, ALPHA)
    slack = lambda a, b: DELTA + 4 * np.spacing(np.maximum(np.abs(a), np.abs(b)))
    assert np.all(np.abs(xp - xl) <= slack(xp, xl))
    assert np.all(np.abs(zp - zl) <= slack(zp, zl))
    assert np.all(xp > 0) and np.all(zp > 0)
    # where no bound binds on the second update, the pair is exactly centred
    free = (np.abs(xp - xl) < DELTA * 0.999) & (np.abs(zp - zl) < DELTA * 0.999)
    assert free.sum() > 100
    assert np.allclose((xp * zp)[free], mu, rtol=1e-12)


def test_reclamp():
    xp = np.array([1e-7, 0.3, 2e-6])
    zp = np.array([0.5, 5e-6, 1e-5])
    a, b = reclamp(xp, zp, 1e-5)
    assert np.array_equal(a, [1e-5, 0.3, 1e-5]) and np.array_equal(b, [0.5, 1e-5, 1e-5])
