"""Interior-point consumer of the centered start (Section 3.1).  TEST INFRASTRUCTURE ONLY.

The paper hands the centered point (x', y, z') of Algorithm 1 to an
interior-point solver and counts its iterations (Section 3.1; Section 4.6,
the iteration-count ratios of its tables).  It uses a commercial barrier
solver and describes no internals, so every choice below is a reading: the
textbook primal-dual method with Mehrotra's predictor-corrector (Wright,
Primal-Dual Interior-Point Methods, 1997, Chapter 10; Mehrotra 1992), written
from that description.

On the scaled LP min c~^T x s.t. A~ x = b~, x >= 0 (A~ = D_r A D_c,
b~ = D_r b, c~ = D_c c, the scaling of the PDHG solve: Algorithm 1 works on
the scaled model), from a point with x, z > 0, each iteration:
  * tests the three relative conditions of Section 2 on the scaled LP
    (||b~ - A~ x|| <= tol (1 + ||b~||), ||c~ - A~^T y - z|| <= tol (1 + ||c~||),
    |c~^T x - b~^T y| <= tol (1 + |c~^T x| + |b~^T y|)) and stops when all hold;
  * forms the normal matrix M = A~ D A~^T, D = X Z^-1, and solves the Newton
    system A~ dx = r_b, A~^T dy + dz = r_c, Z dx + X dz = r_xz through
    M dy = r_b - A~ (Z^-1 r_xz - D r_c), dx = D A~^T dy + Z^-1 r_xz - D r_c,
    dz = r_c - A~^T dy (a dense direct solve here);
  * predictor: r_xz = -X Z e; the largest steps to the boundary
    a_p = min(1, min_{dx_j < 0} -x_j / dx_j), a_d likewise for z; the
    centering parameter sigma = (mu_aff / mu)^3 with mu = x^T z / n and
    mu_aff the same at the predicted point;
  * corrector: r_xz = sigma mu e - X Z e - dX_aff dZ_aff e, the same matrix;
  * steps min(1, eta * step to the boundary) with eta = 0.9995, separately
    for x and for (y, z).
The iteration count is the number of Newton steps taken.  The cold start is
Mehrotra's heuristic point.  The warm start is Algorithm 1 (centering.py);
its loop raises alpha_min tenfold and lifts x', z' to it while the first
step min(a_p, a_d) is below min_step = 1e-6 (Section 3.1 reports that
minimum step length), and runs the method afresh from the lifted point.

Pins (tests/test_oracle_ipm.py): the optimum of planted LPs (closed form) and
scipy's HiGHS, the Newton direction satisfying the linearised KKT system it
is defined by, Mehrotra's point against the minimum-norm solution of
A~ x = b~ (numpy's least squares), hand-built ratio tests, the centering
parameter's hand values, warm starts from a perturbed optimum finishing in a
few iterations, and the recovery loop lifting alpha_min on a start that
touches the boundary.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np
import scipy.sparse as sp

from .centering import center, reclamp


@dataclass
class IpmResult:
    status: int            # 0 optimal, 1 iteration limit, 3 numerical trouble
    iters: int             # Newton steps taken
    x: np.ndarray          # scaled-space iterate
    y: np.ndarray
    z: np.ndarray
    steps: list = field(default_factory=list)  # (a_p, a_d) of each iteration
    mus: list = field(default_factory=list)    # mu = x^T z / n before each iteration
    rel: tuple = (math.nan, math.nan, math.nan)  # the three relative measures at the end


def scaled_lp(A, b, c, d_row, d_col):
    """A~ = D_r A D_c (entries (d_r a) d_c), b~ = D_r b, c~ = D_c c."""
    At = sp.csr_matrix(sp.diags(d_row) @ sp.csr_matrix(A, dtype=np.float64) @ sp.diags(d_col))
    At.sort_indices()
    return At, d_row * np.asarray(b, dtype=np.float64), d_col * np.asarray(c, dtype=np.float64)


def boundary_step(v: np.ndarray, dv: np.ndarray) -> float:
    """Largest a with v + a dv >= 0 (infinite when no component decreases)."""
    neg = dv < 0.0
    return float(np.min(-v[neg] / dv[neg])) if np.any(neg) else math.inf


def centering_sigma(mu_aff: float, mu: float) -> float:
    return (mu_aff / mu) ** 3


def relative_measures(At, bt, ct, x, y, z):
    rp = float(np.linalg.norm(bt - At @ x)) / (1.0 + float(np.linalg.norm(bt)))
    rd = float(np.linalg.norm(ct - At.T @ y - z)) / (1.0 + float(np.linalg.norm(ct)))
    px, dy = float(ct @ x), float(bt @ y)
    return rp, rd, abs(px - dy) / (1.0 + abs(px) + abs(dy))


def newton(At, x, z, r_b, r_c, r_xz, M=None):
    """The Newton direction of the system above (M = A~ D A~^T may be given)."""
    d = x / z
    if M is None:
        M = (At @ sp.diags(d) @ At.T).toarray()
    t = r_xz / z - d * r_c
    dy = np.linalg.solve(M, r_b - At @ t)
    v = At.T @ dy
    return d * v + t, dy, r_c - v


def mehrotra_start(At, bt, ct):
    """Mehrotra's heuristic start: the minimum-norm x of A~ x = b~ and the
    least-squares y of A~^T y ~ c~, shifted to be positive and then balanced."""
    M = (At @ At.T).toarray()
    x = At.T @ np.linalg.solve(M, bt)
    y = np.linalg.solve(M, At @ ct)
    z = ct - At.T @ y
    x = x + max(-1.5 * float(x.min()), 0.0)
    z = z + max(-1.5 * float(z.min()), 0.0)
    xz = float(x @ z)
    return x + 0.5 * xz / float(z.sum()), y, z + 0.5 * xz / float(x.sum())


def ipm(At, bt, ct, start=None, tol: float = 1e-8, max_iter: int = 100, eta: float = 0.9995) -> IpmResult:
    """Mehrotra predictor-corrector from `start` = (x, y, z) (x, z > 0) or
    from Mehrotra's point."""
    x, y, z = (np.array(v, dtype=np.float64) for v in start) if start is not None else mehrotra_start(At, bt, ct)
    n = x.size
    res = IpmResult(1, 0, x, y, z)
    for k in range(max_iter + 1):
        rel = relative_measures(At, bt, ct, x, y, z)
        res.rel = rel
        if not all(math.isfinite(v) for v in rel):
            res.status = 3
            break
        if max(rel) <= tol:
            res.status = 0
            break
        if k == max_iter:
            break
        mu = float(x @ z) / n
        res.mus.append(mu)
        r_b = bt - At @ x
        r_c = ct - At.T @ y - z
        d = x / z
        M = (At @ sp.diags(d) @ At.T).toarray()
        dxa, dya, dza = newton(At, x, z, r_b, r_c, -x * z, M)
        ap = min(1.0, boundary_step(x, dxa))
        ad = min(1.0, boundary_step(z, dza))
        mu_aff = float((x + ap * dxa) @ (z + ad * dza)) / n
        sigma = centering_sigma(mu_aff, mu)
        dx, dy, dz = newton(At, x, z, r_b, r_c, sigma * mu - x * z - dxa * dza, M)
        ap = min(1.0, eta * boundary_step(x, dx))
        ad = min(1.0, eta * boundary_step(z, dz))
        res.steps.append((ap, ad))
        x = x + ap * dx
        y = y + ad * dy
        z = z + ad * dz
        res.iters = k + 1
    res.x, res.y, res.z = x, y, z
    return res


@dataclass
class HybridResult:
    ipm: IpmResult
    alpha_min: float   # the value the run that was kept started from
    lifts: int         # how many times alpha_min was raised
    mu_target: float


def warm_ipm(At, bt, ct, x, y, z, mu_min: float = 1e-6, delta_max: float = 1e-4, alpha_min: float = 1e-6,
             min_step: float = 1e-6, max_lifts: int = 12, tol: float = 1e-8, max_iter: int = 100,
             eta: float = 0.9995) -> HybridResult:
    """Algorithm 1 from a PDHG solution (x, y, z) of the scaled LP, then the
    interior-point method from (x', y, z'), raising alpha_min while the first
    step is below min_step."""
    xp, zp, mu_t = center(x, z, mu_min, delta_max, alpha_min)
    lifts = 0
    while True:
        r = ipm(At, bt, ct, (xp, y, zp), tol, max_iter, eta)
        small = bool(r.steps) and min(r.steps[0]) < min_step
        if not small or lifts >= max_lifts:
            return HybridResult(r, alpha_min, lifts, mu_t)
        alpha_min *= 10.0
        lifts += 1
        xp, zp = reclamp(xp, zp, alpha_min)
