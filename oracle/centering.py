"""Centered start point of Algorithm 1 (Section 3.1).  TEST INFRASTRUCTURE ONLY.

What the map computes, from a PDHG solution (x, y, z) of the scaled LP and
the parameters mu_min, delta_max, alpha_min (Section 3.1 reports 1e-6, 1e-4,
1e-6 as the best settings):

  * mu_target = max(x^T z / n, mu_min), the average complementarity of the
    given point, floored;
  * each pair (x_j, z_j) is raised to at least alpha_min;
  * the member of the pair that is strictly smaller (z when the two are
    equal) is pulled toward mu_target divided by the other member; then the
    other member is pulled toward mu_target divided by the new value of the
    first.  Each pull ends where the target is, or delta_max away from the
    value it started from, whichever is nearer;
  * y is passed through unchanged.

Afterwards, while the interior-point solver cannot take a step, alpha_min
grows tenfold and both vectors are raised to it again (`reclamp`).

Pins (tests/test_oracle_centering.py): hand-computed cases, and invariants
that follow from the definition (moves bounded by delta_max, positivity,
exact centring when the bounds do not bind).
"""
from __future__ import annotations

import numpy as np


def _pull(v: np.ndarray, target: np.ndarray, delta: float) -> np.ndarray:
    """v moved to target, but by at most delta."""
    return np.minimum(np.maximum(target, v - delta), v + delta)


def center(x, z, mu_min: float = 1e-6, delta_max: float = 1e-4, alpha_min: float = 1e-6):
    """Returns (x', z', mu_target) of Algorithm 1's centring map."""
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    mu_t = max(float(x @ z) / x.size, mu_min)
    xl = np.maximum(x, alpha_min)
    zl = np.maximum(z, alpha_min)
    x_moves_first = xl < zl
    first = np.where(x_moves_first, xl, zl)
    second = np.where(x_moves_first, zl, xl)
    first = _pull(first, mu_t / second, delta_max)
    second = _pull(second, mu_t / first, delta_max)
    return np.where(x_moves_first, first, second), np.where(x_moves_first, second, first), mu_t


def reclamp(xp, zp, alpha_min: float):
    """The loop body run while the interior-point step is too small (after
    alpha_min has been multiplied by 10): lift both vectors to alpha_min."""
    return np.maximum(xp, alpha_min), np.maximum(zp, alpha_min)
