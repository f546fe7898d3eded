"""Centered start point of Algorithm 1 (Section 3.1).  TEST INFRASTRUCTURE ONLY.

Input: a PDHG solution (x, y, z) of the scaled LP and the parameters mu_min,
delta_max, alpha_min (Section 3.1 reports 1e-6, 1e-4, 1e-6 as the best
settings).  mu_target is the larger of the average complementarity x^T z / n
of the given point and mu_min.  Every pair (x_j, z_j) is first lifted to at
least alpha_min; then the smaller of the two is moved toward
mu_target / (the other), by at most delta_max, and afterwards the other one
toward mu_target / (the new smaller one), again by at most delta_max.  y is
passed through.  When the interior-point solver cannot take a step,
alpha_min grows tenfold and both vectors are lifted to it again.

Pins (tests/test_oracle_centering.py): hand-computed cases, and invariants
that follow from the definition (moves bounded by delta_max, positivity,
exact centering when the bounds do not bind).
"""
from __future__ import annotations

import numpy as np


def center(x, z, mu_min: float = 1e-6, delta_max: float = 1e-4, alpha_min: float = 1e-6):
    """Returns (x', z', mu_target), element by element as Algorithm 1 states."""
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    n = x.size
    mu_t = max(float(x @ z) / n, mu_min)
    xp = np.empty(n)
    zp = np.empty(n)
    for j in range(n):
        a = max(x[j], alpha_min)
        b = max(z[j], alpha_min)
        if a < b:
            a = min(max(mu_t / b, a - delta_max), a + delta_max)
            b = min(max(mu_t / a, b - delta_max), b + delta_max)
        else:
            b = min(max(mu_t / a, b - delta_max), b + delta_max)
            a = min(max(mu_t / b, a - delta_max), a + delta_max)
        xp[j] = a
        zp[j] = b
    return xp, zp, mu_t


def reclamp(xp, zp, alpha_min: float):
    """The loop body run while the interior-point step is too small (after
    alpha_min has been multiplied by 10): lift both vectors to alpha_min."""
    return np.maximum(xp, alpha_min), np.maximum(zp, alpha_min)
