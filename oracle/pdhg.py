"""Plain float64 restarted PDHG for min c^T x s.t. Ax = b, x >= 0.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU baseline leg; never by the product.

What the paper fixes (and this file follows literally):
  * the primal/dual pair, A is m x n (Section 2, the two programs);
  * r_P = b - A x and r_D = c - A^T y - z (Section 2, residual vectors);
  * the three relative termination tests with inclusive <= (Section 2);
  * scaling by row and column multipliers, results reported on the original,
    unscaled model (Section 2.1; Section 4.3);
  * the maximum-violation metric max(||r_P||_inf, ||r_D||_inf,
    x^T z / (1 + |c^T x|)) on the original model (Section 4.3).

What the paper leaves open: it only says the PDHG used follows cuPDLP+
(Section 4.1).  The iteration below is that family, with every constant a
reading: Ruiz infinity-norm equilibration plus one Pock-Chambolle (alpha = 1)
pass, a constant step eta = safety / sigma_hat from a fixed-length power
iteration, a primal weight omega, reflected Halpern iterations anchored at the
epoch's start, fixed-point-residual restarts with constants 0.2 / 0.8 / 0.36,
exponentially smoothed primal-weight updates at restarts, evaluation every
`eval_every` iterations at the projected point (x_hat, y_hat), and
z = max(c - A^T y, 0).

Pins (tests/test_oracle_*.py): planted optimum (closed form), brute-force
vertex enumeration, scipy's HiGHS on the same LP, the m = 1 simplex LP, the
fixed point of the PDHG operator at the planted optimum, firm
nonexpansiveness of that operator in its metric, the Halpern O(1/k) residual
bound, a dense ten-line Chambolle-Pock loop (reflection 0, Halpern and
restarts off), the KKT gap identity, hand-built termination cases, scaling
invariants, sigma_hat against a dense SVD, hand-built cases at and just past
every bound of the restart rule, the step rule and the initial primal weight
(with a matrix whose power iteration has not settled after 100 iterations),
a restart schedule derived by hand in integer arithmetic, and finite
differences plus a tangent/adjoint dot-product test for the unrolled map.

General form (bounds l <= x <= u and rows of sense =, >= or <=): the paper
notes that practical models carry inequalities and variable bounds, that they
map onto the standard form, and that solvers usually treat them implicitly
(Section 2).  `solve(..., lo=, hi=, sense=)` treats them implicitly: the
primal step projects onto the box, the dual step projects y onto the sign
cone of each row (free, y >= 0 for >= rows, y <= 0 for <= rows), and the
evaluation uses the reduced costs lambda = c - A^T y projected onto the cone
the bounds allow, the primal residual as the violation of each row's sense,
and the dual objective b^T y + sum_j (l_j lambda_j^+ - u_j lambda_j^-).
With l = 0, u = +inf and every row an equality all of these reduce to the
standard-form quantities above.  Pins: scipy's HiGHS on general LPs, a
planted general optimum (closed form and fixed point), the equivalent
standard-form LP built by slack and split variables, and the special case
above reproducing the standard-form run bit for bit.

Infeasibility (a reading; the paper does not treat it): at every evaluation
after the first, the change (d, e) of the evaluated point since the previous
evaluation is tested as a certificate.  For an infeasible or unbounded LP the
PDHG iterates drift along the minimal displacement of the operator, whose
dual part is a Farkas ray and whose primal part a recession direction; for a
solvable LP the change goes to zero.  e certifies primal infeasibility when
its value b^T e + sum_j l_j mu_j^+ - u_j mu_j^- is positive and the norm of
its residual (-A^T e - mu with mu = -A^T e projected onto the bound cones,
and the part of e outside its rows' sign cones) is at most infeas_tol times
that value; d certifies dual infeasibility when c^T d < 0 and the part of
A d outside the rows' recession cones together with the part of d outside
the bounds' recession cones is at most infeas_tol |c^T d|.  Pinned by
scipy's HiGHS classifying the same LPs as infeasible or unbounded.

Primal weight as a PID controller (a variant, off by default): at an
update, with the error e = log(omega) - log(dy/dx), omega becomes
exp(log(omega) - (theta e + ki I + kd (e - e_prev))), I the sum of the errors
of all updates so far including e, e_prev the previous update's error (0 at
the first).  ki = kd = 0 is the smoothing rule above, which is then computed
in its own form.

Restart to the average (a variant, off by default, meant for halpern = 0):
the projected points of the current epoch are averaged with equal weights,
avg = z_hat after the epoch's first iteration and avg <- avg + (z_hat - avg) / j
after its j-th; a restart
then moves the state and the anchor to that average instead of the last
projected point, and the primal-weight update measures the distances of the
average to the old anchor.  The restart tests themselves are unchanged.

Adaptive step with rejection (a variant, off by default: step_rule = 1,
the per-iteration step rule of PDLP, which the cuPDLP family descends from;
Section 4.1 names that family).  It needs plain PDHG (halpern off, reflection
0, restarts to the last point), so that an iterate is the projected point
T(z) of the previous one.  The step starts at 1 / max_ij |A~_ij| (no power
iteration; or a first step the caller gives).  Every iteration is an attempt: with the current eta it forms
z' = T(z) (tau = eta / omega, sigma = eta omega) and the largest step the
move admits, eta_bar = (omega ||x' - x||^2 + ||y' - y||^2 / omega) /
(2 |(y' - y)^T A~ (x' - x)|) (infinite when the product is 0).  The attempt
is accepted when eta <= eta_bar (z <- z'), rejected otherwise (z stays);
either way the next attempt uses eta <- min((1 - (t + 1)^-0.3) eta_bar,
(1 + (t + 1)^-0.6) eta), t the attempt's 1-based number.  Readings: t counts
every attempt, rejected ones included, and so do the iteration limit, the
evaluation schedule and the restart rule's k and t; the fixed-point residual
R of an evaluation is that of its attempt, z - T(z) with the attempt's step,
while the evaluated and restart point is the current z (after the accept or
reject).  Pinned by hand-built accept, reject and boundary cases of the rule,
the bound |dy^T A~ dx| <= ||A~||_2 ||dz||^2_omega / 2 (a step of at most
1 / ||A~||_2 is never rejected, whatever the move), planted optima reached
with rejections on the way, and rejected attempts leaving the iterate
unchanged.

The restart rule, the primal-weight update and the step rule are pinned as
definitions (hand-built cases above).  What no pin can fix is whether these
constants are those of the solver the paper used: the iteration counts to a
tolerance that follow from them are this reading's, compared GPU against
oracle only.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np
import scipy.sparse as sp

STATUS = {0: "OPTIMAL", 1: "ITER_LIMIT", 2: "TIME_LIMIT", 3: "NUMERICAL", 4: "PRIMAL_INFEASIBLE",
          5: "DUAL_INFEASIBLE"}
SENSE_EQ, SENSE_GE, SENSE_LE = 0, 1, 2  # (A x)_i = b_i, >= b_i, <= b_i


@dataclass
class OracleOptions:
    ruiz_iters: int = 10
    pock_chambolle: bool = True
    power_iters: int = 100
    eval_every: int = 64
    step_safety: float = 0.95
    reflect_rho: float = 1.0
    halpern: bool = True
    restarts: bool = True
    beta_suff: float = 0.2
    beta_nec: float = 0.8
    beta_art: float = 0.36
    pw_theta: float = 0.5
    max_iter: int = 1_000_000
    infeas_tol: float = 1e-8  # 0 turns the certificate tests off
    pw_ki: float = 0.0        # primal weight as a PID controller: integral gain
    pw_kd: float = 0.0        # and derivative gain (pw_theta is the proportional one)
    restart_avg: bool = False  # restart to the epoch's average of the projected points
    step_rule: int = 0         # 0: eta = safety / sigma_hat; 1: adaptive with rejection (plain PDHG only)
    step0: float = 0.0         # step_rule 1: the first step (0: 1 / max |A~_ij|)


@dataclass
class Measures:
    """Quantities of Section 2 and Section 4.3, on the original model."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    r_p: np.ndarray
    r_d: np.ndarray
    rp_norm: float
    rd_norm: float
    pobj: float
    dobj: float
    gap: float
    rp_inf: float
    rd_inf: float
    xz: float
    violation: float


@dataclass
class Result:
    status: int
    iters: int
    restarts: int
    meas: Measures
    d_row: np.ndarray
    d_col: np.ndarray
    sigma_hat: float
    eta: float
    omega0: float
    omega: float
    log: list = field(default_factory=list)  # (t, restarted, omega after)
    trace: dict = field(default_factory=dict)  # t -> (x, y, x_hat, y_hat), scaled
    evals: list = field(default_factory=list)  # (t, k, R, R0, R_prev) seen by each restart decision
    rejected: int = 0  # step_rule 1: attempts whose step was rejected


# ---------------------------------------------------------------------------
# input validation (the standard form of Section 2)
# ---------------------------------------------------------------------------

def validate_general(n: int, m: int, lo, hi, sense) -> None:
    """Bounds: no NaN, l < +inf, u > -inf, l <= u; senses in {0, 1, 2}."""
    if lo.shape != (n,) or hi.shape != (n,) or sense.shape != (m,):
        raise ValueError("shape mismatch")
    if np.any(np.isnan(lo)) or np.any(np.isnan(hi)):
        raise ValueError("NaN bound")
    if np.any(lo == np.inf) or np.any(hi == -np.inf) or np.any(lo > hi):
        raise ValueError("empty bound interval")
    if np.any((sense < 0) | (sense > 2)):
        raise ValueError("row sense must be 0, 1 or 2")


def validate(A: sp.csr_matrix, AT: sp.csr_matrix, b: np.ndarray, c: np.ndarray) -> None:
    """Shapes, finiteness, and that AT is exactly the transpose of A."""
    m, n = A.shape
    if m < 1 or n < 1:
        raise ValueError("empty LP")
    if AT.shape != (n, m) or b.shape != (m,) or c.shape != (n,):
        raise ValueError("shape mismatch")
    for v in (A.data, AT.data, b, c):
        if not np.all(np.isfinite(v)):
            raise ValueError("non-finite input")
    own = sp.csr_matrix(A.T)
    own.sort_indices()
    other = AT.copy()
    other.sort_indices()
    if own.nnz != other.nnz or abs(own - other).max() != 0.0:
        raise ValueError("AT is not the transpose of A")


# ---------------------------------------------------------------------------
# scaling (Section 2.1; equilibration + Pock-Chambolle is a reading)
# ---------------------------------------------------------------------------

def _inv_sqrt_or_one(v: np.ndarray) -> np.ndarray:
    out = np.ones_like(v)
    pos = v > 0
    out[pos] = 1.0 / np.sqrt(v[pos])
    return out


def scale(A: sp.csr_matrix, ruiz_iters: int = 10, pock_chambolle: bool = True):
    """Row/column multipliers D_r, D_c and the scaled matrix D_r A D_c.

    Each Ruiz pass takes every row's and every column's largest |entry| of the
    current scaled matrix and divides the row/column by the square root of it
    (factor 1 for an empty row or column).  The optional last pass does the
    same with row and column sums of |entries| (Pock-Chambolle, alpha = 1),
    which bounds the spectral norm of the result by 1.
    """
    At = sp.csr_matrix(A, dtype=np.float64, copy=True)
    m, n = At.shape
    d_row = np.ones(m)
    d_col = np.ones(n)

    def one_pass(row_stat: np.ndarray, col_stat: np.ndarray):
        nonlocal At, d_row, d_col
        r = _inv_sqrt_or_one(row_stat)
        s = _inv_sqrt_or_one(col_stat)
        At = sp.csr_matrix(sp.diags(r) @ At @ sp.diags(s))
        d_row = d_row * r
        d_col = d_col * s

    for _ in range(ruiz_iters):
        absA = abs(At)
        one_pass(np.asarray(absA.max(axis=1).todense()).ravel(),
                 np.asarray(absA.max(axis=0).todense()).ravel())
    if pock_chambolle:
        absA = abs(At)
        one_pass(np.asarray(absA.sum(axis=1)).ravel(),
                 np.asarray(absA.sum(axis=0)).ravel())
    At.sort_indices()
    return d_row, d_col, At


# ---------------------------------------------------------------------------
# step size and primal weight (readings of the cuPDLP+ family, Section 4.1)
# ---------------------------------------------------------------------------

def power_sigma(At: sp.csr_matrix, iters: int = 100):
    """Largest singular value of At by `iters` power iterations on At^T At from
    the unit vector 1/sqrt(n).  Returns (sigma_hat, history) where history[k]
    is ||At v_k|| for the k-th normalised iterate (history[-1] = sigma_hat)."""
    n = At.shape[1]
    v = np.full(n, 1.0 / math.sqrt(n))
    hist = []
    for _ in range(iters):
        Av = At @ v
        hist.append(float(np.linalg.norm(Av)))
        u = At.T @ Av
        nu = float(np.linalg.norm(u))
        if nu == 0.0:
            break
        v = u / nu
    sigma = float(np.linalg.norm(At @ v))
    hist.append(sigma)
    return sigma, hist


def step_size(sigma_hat: float, hist: list, opts: OracleOptions) -> float:
    """eta = safety / sigma_hat, unless the power iteration has not settled
    (relative change over its last 10 iterations above 1e-3) and the
    Pock-Chambolle pass guarantees ||At||_2 <= 1, in which case eta = safety."""
    if sigma_hat <= 0.0:
        return opts.step_safety
    if opts.pock_chambolle and len(hist) > 10:
        if abs(hist[-1] - hist[-11]) > 1e-3 * hist[-1]:
            return opts.step_safety
    return opts.step_safety / sigma_hat


def adaptive_initial_step(At) -> float:
    """step_rule 1: the first step, 1 / (largest |entry| of the scaled matrix)."""
    big = float(np.max(np.abs(At.data))) if At.nnz else 0.0
    return 1.0 / big if big > 0.0 else 1.0


def adaptive_step(dx2: float, dy2: float, cross: float, eta: float, omega: float, t: int):
    """step_rule 1 on one attempt of step eta, whose move has squared norms
    dx2 = ||x' - x||^2, dy2 = ||y' - y||^2 and cross = (y' - y)^T A~ (x' - x):
    returns (accepted, next step, eta_bar)."""
    mag = abs(cross)
    eta_bar = (omega * dx2 + dy2 / omega) / (2.0 * mag) if mag > 0.0 else math.inf
    nxt = min((1.0 - (t + 1.0) ** -0.3) * eta_bar, (1.0 + (t + 1.0) ** -0.6) * eta)
    return eta <= eta_bar, nxt, eta_bar


def initial_weight(bt: np.ndarray, ct: np.ndarray) -> float:
    nb = float(np.linalg.norm(bt))
    nc = float(np.linalg.norm(ct))
    if nb > 1e-10 and nc > 1e-10:
        return nc / nb
    return 1.0


# ---------------------------------------------------------------------------
# the PDHG operator on the scaled problem
# ---------------------------------------------------------------------------

def pdhg_operator(At, AtT, bt, ct, tau, sig, x, y, lo_t=None, hi_t=None, sense=None):
    """One PDHG step T(x, y) = (x_hat, y_hat) for the saddle problem
    min_{x in X} max_{y in Y} c^T x - y^T (A x - b): a projected primal
    gradient step, then a dual ascent step at the extrapolated point
    2 x_hat - x.  Standard form: X = {x >= 0}, Y = R^m.  General form:
    X = [lo_t, hi_t] (scaled bounds), Y_i = R, [0, inf) or (-inf, 0] for rows
    of sense =, >= or <= (the Lagrangian term y_i (b_i - (A x)_i) is bounded
    above over Y_i exactly when row i holds)."""
    g = ct - AtT @ y
    if lo_t is None:
        x_hat = np.maximum(x - tau * g, 0.0)
    else:
        x_hat = np.minimum(np.maximum(x - tau * g, lo_t), hi_t)
    x_bar = 2.0 * x_hat - x
    y_hat = y + sig * (bt - At @ x_bar)
    if sense is not None:
        ge, le = sense == SENSE_GE, sense == SENSE_LE
        y_hat[ge] = np.maximum(y_hat[ge], 0.0)
        y_hat[le] = np.minimum(y_hat[le], 0.0)
    return x_hat, y_hat


# ---------------------------------------------------------------------------
# evaluation on the original model (Section 2 tests; Section 4.3 metric)
# ---------------------------------------------------------------------------

def reduced_costs(g: np.ndarray, lo, hi) -> np.ndarray:
    """lambda = g projected onto the cone the bounds allow: R where both bounds
    are finite, [0, inf) with only a lower bound, (-inf, 0] with only an upper
    bound, {0} for a free variable (standard form: z = max(g, 0))."""
    if lo is None:
        return np.maximum(g, 0.0)
    lf, uf = np.isfinite(lo), np.isfinite(hi)
    return np.where(lf & uf, g, np.where(lf, np.maximum(g, 0.0), np.where(uf, np.minimum(g, 0.0), 0.0)))


def evaluate(A, AT, b, c, d_row, d_col, x_hat, y_hat, lo=None, hi=None, sense=None) -> Measures:
    x = d_col * x_hat
    y = d_row * y_hat
    Ax = A @ x
    ATy = AT @ y
    z = reduced_costs(c - ATy, lo, hi)
    r_p = b - Ax
    if sense is not None:  # a row's residual is its violation
        r_p = np.where(sense == SENSE_GE, np.maximum(r_p, 0.0),
                       np.where(sense == SENSE_LE, np.minimum(r_p, 0.0), r_p))
    r_d = c - ATy - z
    pobj = float(c @ x)
    dobj = float(b @ y)
    if lo is None:
        xz = float(x @ z)
    else:  # bound terms of the dual objective; complementarity with the bounds
        lf, uf = np.isfinite(lo), np.isfinite(hi)
        lo0, hi0 = np.where(lf, lo, 0.0), np.where(uf, hi, 0.0)  # lambda is 0 where a bound is infinite
        zp, zm = np.maximum(z, 0.0), np.maximum(-z, 0.0)
        dobj += float(np.sum(lo0 * zp) - np.sum(hi0 * zm))
        xz = float(np.sum(np.where(lf, zp * (x - lo0), 0.0)) + np.sum(np.where(uf, zm * (hi0 - x), 0.0)))
    rp_inf = float(np.abs(r_p).max()) if r_p.size else 0.0
    rd_inf = float(np.abs(r_d).max()) if r_d.size else 0.0
    return Measures(x, y, z, r_p, r_d, float(np.linalg.norm(r_p)), float(np.linalg.norm(r_d)),
                    pobj, dobj, abs(pobj - dobj), rp_inf, rd_inf, xz,
                    max(rp_inf, rd_inf, xz / (1.0 + abs(pobj))))


def ray_measures(A, AT, b, c, d, e, lo=None, hi=None, sense=None):
    """Certificate quantities of a direction pair in the original space:
    (value of e as a dual ray, its residual norm, c^T d, residual norm of d as
    a primal ray); see the module docstring."""
    Ad = A @ d
    g = -(AT @ e)
    mu = reduced_costs(g, lo, hi)
    if sense is None:
        viol_ad, viol_e = Ad, np.zeros(0)
    else:
        ge, le = sense == SENSE_GE, sense == SENSE_LE
        viol_ad = np.where(ge, np.minimum(Ad, 0.0), np.where(le, np.maximum(Ad, 0.0), Ad))
        viol_e = np.where(ge, np.minimum(e, 0.0), np.where(le, np.maximum(e, 0.0), 0.0))
    if lo is None:
        bterm = 0.0
        viol_d = np.minimum(d, 0.0)
    else:
        lf, uf = np.isfinite(lo), np.isfinite(hi)
        lo0, hi0 = np.where(lf, lo, 0.0), np.where(uf, hi, 0.0)
        bterm = float(np.sum(lo0 * np.maximum(mu, 0.0)) - np.sum(hi0 * np.maximum(-mu, 0.0)))
        viol_d = np.where(lf & uf, d, np.where(lf, np.minimum(d, 0.0), np.where(uf, np.maximum(d, 0.0), 0.0)))
    q_e = float(b @ e) + bterm
    r_e = math.sqrt(float(np.sum((g - mu) ** 2)) + float(np.sum(viol_e ** 2)))
    q_d = float(c @ d)
    r_d = math.sqrt(float(np.sum(viol_ad ** 2)) + float(np.sum(viol_d ** 2)))
    return q_e, r_e, q_d, r_d


def infeasibility(q_e: float, r_e: float, q_d: float, r_d: float, tol: float):
    """4 (primal infeasible), 5 (dual infeasible) or None."""
    if tol <= 0.0:
        return None
    if q_e > 0.0 and r_e <= tol * q_e:
        return 4
    if q_d < 0.0 and r_d <= tol * -q_d:
        return 5
    return None


def terminated(meas: Measures, b_norm: float, c_norm: float, eps: float) -> bool:
    """The three relative tests of Section 2, inclusive."""
    return (meas.rp_norm <= eps * (1.0 + b_norm)
            and meas.rd_norm <= eps * (1.0 + c_norm)
            and meas.gap <= eps * (1.0 + abs(meas.pobj) + abs(meas.dobj)))


def primal_weight_update(omega: float, dx: float, dy: float, pid: list, opts: OracleOptions) -> float:
    """The primal weight after a restart whose distances to the epoch's anchor
    are dx, dy (both > 1e-10); pid = [integral, previous error, count] is
    updated in place."""
    th = opts.pw_theta
    if opts.pw_ki == 0.0 and opts.pw_kd == 0.0:
        return math.exp(th * math.log(dy / dx) + (1.0 - th) * math.log(omega))
    e = math.log(omega) - math.log(dy / dx)
    pid[0] += e
    de = e - pid[1] if pid[2] > 0 else 0.0
    pid[1] = e
    pid[2] += 1
    return math.exp(math.log(omega) - (th * e + opts.pw_ki * pid[0] + opts.pw_kd * de))


def restart_due(R: float, R0: float, R_prev: float, k: int, t: int, opts: OracleOptions) -> bool:
    """Sufficient decay, necessary decay without progress, or an epoch that
    has grown past a fixed share of all iterations (k counts this iteration)."""
    if R <= opts.beta_suff * R0:
        return True
    if R <= opts.beta_nec * R0 and R > R_prev:
        return True
    return float(k) >= opts.beta_art * float(t)


# ---------------------------------------------------------------------------
# the solve loop
# ---------------------------------------------------------------------------

def solve(A, AT, b, c, eps: float, opts: OracleOptions | None = None,
          x_init=None, y_init=None, trace_iters: int = 0, lo=None, hi=None, sense=None) -> Result:
    """Standard form, or the general form when any of lo, hi, sense is given
    (missing ones default to 0, +inf and all equalities)."""
    opts = opts or OracleOptions()
    A = sp.csr_matrix(A)
    AT = sp.csr_matrix(AT)
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    validate(A, AT, b, c)
    m, n = A.shape
    general = lo is not None or hi is not None or sense is not None
    if general:
        lo = np.zeros(n) if lo is None else np.asarray(lo, dtype=np.float64)
        hi = np.full(n, np.inf) if hi is None else np.asarray(hi, dtype=np.float64)
        sense = np.zeros(m, dtype=np.int8) if sense is None else np.asarray(sense, dtype=np.int8)
        validate_general(n, m, lo, hi, sense)
    b_norm = float(np.linalg.norm(b))
    c_norm = float(np.linalg.norm(c))

    d_row, d_col, At = scale(A, opts.ruiz_iters, opts.pock_chambolle)
    AtT = sp.csr_matrix(At.T)
    bt = d_row * b
    ct = d_col * c
    lo_t = lo / d_col if general else None
    hi_t = hi / d_col if general else None
    adaptive = opts.step_rule == 1
    if adaptive:
        if opts.halpern or opts.reflect_rho != 0.0 or opts.restart_avg:
            raise ValueError("step_rule 1 needs halpern off, reflect_rho 0 and restarts to the last point")
        sigma_hat, eta = 0.0, (opts.step0 if opts.step0 > 0.0 else adaptive_initial_step(At))
    else:
        sigma_hat, hist = power_sigma(At, opts.power_iters)
        eta = step_size(sigma_hat, hist, opts)
    rejected = 0
    omega0 = initial_weight(bt, ct)
    omega = omega0
    tau, sig = eta / omega, eta * omega

    x = np.zeros(n) if x_init is None else np.asarray(x_init, dtype=np.float64) / d_col
    y = np.zeros(m) if y_init is None else np.asarray(y_init, dtype=np.float64) / d_row
    x0, y0 = x.copy(), y.copy()
    rho = opts.reflect_rho
    k = 0
    t = 0
    R0 = math.nan
    R_prev = math.inf
    restarts = 0
    log = []
    evals = []
    trace = {}
    E = max(1, int(opts.eval_every))
    prev = None  # the previous evaluated point (x, y), original space
    pid = [0.0, 0.0, 0]  # primal-weight controller state
    x_avg, y_avg = np.zeros(n), np.zeros(m)  # epoch averages (restart_avg)

    while True:
        t += 1
        x_hat, y_hat = pdhg_operator(At, AtT, bt, ct, tau, sig, x, y, lo_t, hi_t, sense)
        R = math.sqrt(omega * float(np.sum((x - x_hat) ** 2))
                      + float(np.sum((y - y_hat) ** 2)) / omega)
        if k == 0:
            R0 = R
        if adaptive:  # accept T(z) or keep z; either way the step changes
            dx, dy = x_hat - x, y_hat - y
            ok, eta, _ = adaptive_step(float(dx @ dx), float(dy @ dy), float(dy @ (At @ dx)), eta, omega, t)
            tau, sig = eta / omega, eta * omega
            x_new, y_new = (x_hat, y_hat) if ok else (x.copy(), y.copy())
            rejected += 0 if ok else 1
            x_ev, y_ev = x_new, y_new
        else:
            w = (k + 1.0) / (k + 2.0) if opts.halpern else 1.0
            x_new = w * ((1.0 + rho) * x_hat - rho * x) + (1.0 - w) * x0
            y_new = w * ((1.0 + rho) * y_hat - rho * y) + (1.0 - w) * y0
            x_ev, y_ev = x_hat, y_hat
        if opts.restart_avg:  # the mean of the epoch's points; the first is its own mean
            if k == 0:
                x_avg, y_avg = x_hat.copy(), y_hat.copy()
            else:
                inv = 1.0 / (k + 1.0)
                x_avg = x_avg + (x_hat - x_avg) * inv
                y_avg = y_avg + (y_hat - y_avg) * inv
        k += 1
        restarted = False
        if t % E == 0 or t == opts.max_iter:
            meas = evaluate(A, AT, b, c, d_row, d_col, x_ev, y_ev, lo, hi, sense)
            status = None
            if not all(math.isfinite(v) for v in (meas.rp_norm, meas.rd_norm, meas.pobj, meas.dobj)):
                status = 3
            elif terminated(meas, b_norm, c_norm, eps):
                status = 0
            if status is None and prev is not None:
                status = infeasibility(*ray_measures(A, AT, b, c, meas.x - prev[0], meas.y - prev[1],
                                                     lo, hi, sense), opts.infeas_tol)
            if status is None and t >= opts.max_iter:
                status = 1
            if status is not None:
                if t <= trace_iters:
                    trace[t] = (x_new, y_new, x_ev, y_ev)
                return Result(status, t, restarts, meas, d_row, d_col, sigma_hat, eta,
                              omega0, omega, log, trace, evals, rejected)
            evals.append((t, k, R, R0, R_prev))
            if opts.restarts and restart_due(R, R0, R_prev, k, t, opts):
                px, py = (x_avg, y_avg) if opts.restart_avg else (x_ev, y_ev)
                dx = float(np.linalg.norm(px - x0))
                dy = float(np.linalg.norm(py - y0))
                if dx > 1e-10 and dy > 1e-10:
                    omega = primal_weight_update(omega, dx, dy, pid, opts)
                    tau, sig = eta / omega, eta * omega
                x_new, y_new = px.copy(), py.copy()
                x0, y0 = px.copy(), py.copy()
                k = 0
                R_prev = math.inf
                restarts += 1
                restarted = True
            else:
                R_prev = R
            log.append((t, restarted, omega))
            prev = (meas.x, meas.y)
        x, y = x_new, y_new
        if t <= trace_iters:
            trace[t] = (x.copy(), y.copy(), x_ev, y_ev)


# ---------------------------------------------------------------------------
# the differentiable unrolled map: exactly K iterations, schedule frozen
# ---------------------------------------------------------------------------

@dataclass
class Schedule:
    """Restart iterations and the (tau, sigma) of every epoch, recorded by a
    forward run and replayed unchanged by perturbed runs."""
    restart_at: list
    taus: list
    sigmas: list


@dataclass
class _Prep:
    d_row: np.ndarray
    d_col: np.ndarray
    At: sp.csr_matrix
    AtT: sp.csr_matrix
    eta: float


def _prepare(A, opts: OracleOptions) -> _Prep:
    d_row, d_col, At = scale(sp.csr_matrix(A), opts.ruiz_iters, opts.pock_chambolle)
    sigma_hat, hist = power_sigma(At, opts.power_iters)
    return _Prep(d_row, d_col, At, sp.csr_matrix(At.T), step_size(sigma_hat, hist, opts))


def unrolled_forward(A, b, c, K: int, opts: OracleOptions | None = None,
                     schedule: Schedule | None = None, keep_masks: bool = False,
                     prep: _Prep | None = None):
    """x_K = D_c x_hat_K after exactly K iterations from (0, 0).

    Without a schedule, restarts are decided by the usual rule at evaluation
    points (no termination test) and recorded; with one, its restart
    iterations and per-epoch steps are used as constants."""
    opts = opts or OracleOptions()
    p = prep or _prepare(A, opts)
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    bt = p.d_row * b
    ct = p.d_col * c
    m, n = p.At.shape
    if schedule is None:
        omega = initial_weight(bt, ct)
        rec = Schedule([], [p.eta / omega], [p.eta * omega])
    else:
        omega = math.nan
        rec = schedule
    epoch = 0
    tau, sig = rec.taus[0], rec.sigmas[0]
    restart_set = set(rec.restart_at) if schedule is not None else None
    x = np.zeros(n)
    y = np.zeros(m)
    x0, y0 = x.copy(), y.copy()
    rho = opts.reflect_rho
    k = 0
    R0 = math.nan
    R_prev = math.inf
    masks = []
    ws = []
    restart_flags = []
    x_hat = x
    E = max(1, int(opts.eval_every))
    for t in range(1, K + 1):
        g = ct - p.AtT @ y
        v = x - tau * g
        x_hat = np.maximum(v, 0.0)
        if keep_masks:
            masks.append(v > 0.0)
        x_bar = 2.0 * x_hat - x
        y_hat = y + sig * (bt - p.At @ x_bar)
        w = (k + 1.0) / (k + 2.0) if opts.halpern else 1.0
        ws.append(w)
        if schedule is None:
            R = math.sqrt(omega * float(np.sum((x - x_hat) ** 2))
                          + float(np.sum((y - y_hat) ** 2)) / omega)
            if k == 0:
                R0 = R
        k += 1
        do_restart = False
        if t < K and t % E == 0:
            if schedule is None:
                if opts.restarts and restart_due(R, R0, R_prev, k, t, opts):
                    do_restart = True
                    dx = float(np.linalg.norm(x_hat - x0))
                    dy = float(np.linalg.norm(y_hat - y0))
                    if dx > 1e-10 and dy > 1e-10:
                        th = opts.pw_theta
                        omega = math.exp(th * math.log(dy / dx) + (1.0 - th) * math.log(omega))
                    rec.restart_at.append(t)
                    rec.taus.append(p.eta / omega)
                    rec.sigmas.append(p.eta * omega)
                    R_prev = math.inf
                else:
                    R_prev = R
            else:
                do_restart = t in restart_set
        restart_flags.append(do_restart)
        if do_restart:
            epoch += 1
            tau, sig = rec.taus[epoch], rec.sigmas[epoch]
            x, y = x_hat.copy(), y_hat.copy()
            x0, y0 = x_hat.copy(), y_hat.copy()
            k = 0
        else:
            x = w * ((1.0 + rho) * x_hat - rho * x) + (1.0 - w) * x0
            y = w * ((1.0 + rho) * y_hat - rho * y) + (1.0 - w) * y0
    x_K = p.d_col * x_hat
    tape = {"masks": masks, "ws": ws, "restart": restart_flags, "prep": p}
    return x_K, rec, tape


def unrolled_grad(A, b, c, K: int, wvec, opts: OracleOptions | None = None,
                  schedule: Schedule | None = None):
    """Reverse mode of the unrolled map for the loss w^T x_K.

    Walks the iterations backwards with the recorded projection masks
    1[x - tau g > 0] (0 at exactly 0) and returns (dL/dc, dL/db, x_K, schedule).
    """
    opts = opts or OracleOptions()
    x_K, sched, tape = unrolled_forward(A, b, c, K, opts, schedule, keep_masks=True)
    p = tape["prep"]
    m, n = p.At.shape
    rho = opts.reflect_rho
    # per-iteration (tau, sigma) from the schedule
    taus, sigs = [], []
    epoch = 0
    for t in range(1, K + 1):
        taus.append(sched.taus[epoch])
        sigs.append(sched.sigmas[epoch])
        if tape["restart"][t - 1]:
            epoch += 1
    lx = np.zeros(n)   # adjoint of the state x after iteration t
    ly = np.zeros(m)
    lx0 = np.zeros(n)  # adjoint of the anchor after iteration t
    ly0 = np.zeros(m)
    lct = np.zeros(n)
    lbt = np.zeros(m)
    seed = p.d_col * np.asarray(wvec, dtype=np.float64)
    for t in range(K, 0, -1):
        i = t - 1
        w = tape["ws"][i]
        if tape["restart"][i]:
            lxh = lx + lx0
            lyh = ly + ly0
            lx_prev = np.zeros(n)
            ly_prev = np.zeros(m)
            lx0_prev = np.zeros(n)
            ly0_prev = np.zeros(m)
        else:
            lxh = w * (1.0 + rho) * lx
            lyh = w * (1.0 + rho) * ly
            lx_prev = -w * rho * lx
            ly_prev = -w * rho * ly
            lx0_prev = lx0 + (1.0 - w) * lx
            ly0_prev = ly0 + (1.0 - w) * ly
        if t == K:
            lxh = lxh + seed
        # y_hat = y + sigma (bt - At x_bar)
        ly_prev = ly_prev + lyh
        lbt += sigs[i] * lyh
        lxbar = -sigs[i] * (p.AtT @ lyh)
        # x_bar = 2 x_hat - x
        lxh = lxh + 2.0 * lxbar
        lx_prev = lx_prev - lxbar
        # x_hat = max(v, 0), v = x - tau g, g = ct - At^T y
        lv = np.where(tape["masks"][i], lxh, 0.0)
        lx_prev = lx_prev + lv
        lg = -taus[i] * lv
        lct += lg
        ly_prev = ly_prev - p.At @ lg
        lx, ly, lx0, ly0 = lx_prev, ly_prev, lx0_prev, ly0_prev
    return p.d_col * lct, p.d_row * lbt, x_K, sched


def unrolled_tangent(A, b, c, K: int, dc, db, opts: OracleOptions | None = None,
                     schedule: Schedule | None = None):
    """Forward-mode derivative of x_K along (dc, db) with the masks and the
    schedule of the unperturbed run."""
    opts = opts or OracleOptions()
    x_K, sched, tape = unrolled_forward(A, b, c, K, opts, schedule, keep_masks=True)
    p = tape["prep"]
    m, n = p.At.shape
    rho = opts.reflect_rho
    dbt = p.d_row * np.asarray(db, dtype=np.float64)
    dct = p.d_col * np.asarray(dc, dtype=np.float64)
    dx = np.zeros(n)
    dy = np.zeros(m)
    dx0 = dx.copy()
    dy0 = dy.copy()
    epoch = 0
    dxh = dx
    for t in range(1, K + 1):
        i = t - 1
        tau, sig = sched.taus[epoch], sched.sigmas[epoch]
        dg = dct - p.AtT @ dy
        dv = dx - tau * dg
        dxh = np.where(tape["masks"][i], dv, 0.0)
        dxbar = 2.0 * dxh - dx
        dyh = dy + sig * (dbt - p.At @ dxbar)
        w = tape["ws"][i]
        if tape["restart"][i]:
            epoch += 1
            dx, dy = dxh.copy(), dyh.copy()
            dx0, dy0 = dxh.copy(), dyh.copy()
        else:
            dx = w * ((1.0 + rho) * dxh - rho * dx) + (1.0 - w) * dx0
            dy = w * ((1.0 + rho) * dyh - rho * dy) + (1.0 - w) * dy0
    return p.d_col * dxh, x_K, sched
