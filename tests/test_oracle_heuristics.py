"""Pins of the oracle's step, primal-weight start and restart rule.

The paper leaves these internals to the cuPDLP+ family it cites (Section 4.1);
their readings are: eta = safety / sigma_hat unless the power iteration has
not settled (then eta = safety, which the Pock-Chambolle pass makes safe),
omega_0 = ||c~|| / ||b~|| with a fallback of 1, and a restart at an evaluation
when R <= beta_suff R0, or R <= beta_nec R0 while R grew since the previous
evaluation, or the epoch holds at least beta_art of all iterations.

Each expected value below is written out by hand from those definitions
(threshold cases exactly at and just beyond each bound, a schedule of
artificial restarts derived in integer arithmetic, scaling factors of a 1 x 2
matrix worked on paper), or comes from a dense SVD, HiGHS, or a ten-line
dense Chambolle-Pock loop that shares nothing with the oracle.
"""
import math

import numpy as np
import pytest
import scipy.optimize
import scipy.sparse as sp

import lpgen
import oracle
from oracle.pdhg import OracleOptions, initial_weight, restart_due, step_size

INF = math.inf
up = lambda v: math.nextafter(v, INF)      # noqa: E731
down = lambda v: math.nextafter(v, -INF)   # noqa: E731


# ---------------------------------------------------------------------------
# restart rule: each criterion at and just beyond its bound
# ---------------------------------------------------------------------------

D = OracleOptions()  # 0.2 / 0.8 / 0.36


@pytest.mark.parametrize("R,R0,R_prev,k,t,expected", [
    # sufficient decay, inclusive: 0.2 * 10 = 2 exactly
    (2.0, 10.0, INF, 1, 100, True),
    (up(2.0), 10.0, INF, 1, 100, False),
    (1.0, 10.0, 0.5, 1, 100, True),            # sufficient decay needs no growth
    # necessary decay with growth, inclusive: 0.8 * 10 = 8 exactly
    (8.0, 10.0, 7.0, 1, 100, True),
    (up(8.0), 10.0, 7.0, 1, 100, False),
    (5.0, 10.0, down(5.0), 1, 100, True),      # grew by one ulp
    (5.0, 10.0, 5.0, 1, 100, False),           # equal is no growth
    (5.0, 10.0, 6.0, 1, 100, False),           # still shrinking
    (5.0, 10.0, INF, 1, 100, False),           # first evaluation of an epoch
    # artificial: k >= 0.36 t, k counting the current iteration
    (9.5, 10.0, 1.0, 36, 100, True),
    (9.5, 10.0, 1.0, 35, 100, False),
    (9.5, 10.0, 1.0, 9, 25, True),
    (9.5, 10.0, 1.0, 8, 25, False),
    (9.5, 10.0, 1.0, 24, 64, True),            # 0.36 * 64 = 23.04
    (9.5, 10.0, 1.0, 23, 64, False),
    (9.5, 10.0, 1.0, 64, 64, True),            # the first evaluation of a solve
    # nothing holds
    (9.5, 10.0, 9.0, 1, 100, False),
])
def test_restart_due_default_constants(R, R0, R_prev, k, t, expected):
    assert restart_due(R, R0, R_prev, k, t, D) is expected


@pytest.mark.parametrize("R,R_prev,k,t,expected", [
    (1.0, INF, 1, 100, True),          # 0.1 * 10 = 1
    (1.5, INF, 1, 100, False),         # would pass at 0.2
    (9.0, 8.0, 1, 100, True),          # 0.9 * 10 = 9, and grew
    (up(9.0), 8.0, 1, 100, False),
    (9.5, 1.0, 50, 100, True),         # 0.5 * 100 = 50
    (9.5, 1.0, 49, 100, False),        # would pass at 0.36
])
def test_restart_due_custom_constants(R, R_prev, k, t, expected):
    """Other constants take each criterion's own place (a swap of two of
    them, or a constant hard-coded in place of its option, fails here)."""
    o = OracleOptions(beta_suff=0.1, beta_nec=0.9, beta_art=0.5)
    assert restart_due(R, 10.0, R_prev, k, t, o) is expected


def _restart_iters(res):
    return [t for t, r, _ in res.log if r]


@pytest.mark.parametrize("E,max_iter,expected", [
    # only the artificial criterion can fire (beta_suff = beta_nec = 0 need
    # R = 0).  A restart at evaluation t after one at t0 needs
    # 100 (t - t0) >= 36 t, i.e. t >= 1.5625 t0:
    (1, 120, [1, 2, 4, 7, 11, 18, 29, 46, 72, 113]),
    # the same at multiples of 64: 64, then t >= 100 -> 128, t >= 200 -> 256,
    # t >= 400 -> 448, t >= 700 -> 704
    (64, 1000, [64, 128, 256, 448, 704]),
])
def test_artificial_restart_schedule(E, max_iter, expected):
    lp = lpgen.cfg1(0)
    o = OracleOptions(beta_suff=0.0, beta_nec=0.0, eval_every=E, max_iter=max_iter, infeas_tol=0.0)
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-30, opts=o)
    assert res.status == 1
    assert _restart_iters(res) == expected


def test_restart_bookkeeping_every_iteration():
    """With an evaluation every iteration, every decision's inputs can be
    followed: k counts the epoch's iterations including the current one, R0
    is R of the epoch's first iteration, R_prev is the previous evaluation's R
    within an epoch and +inf at its first, and the state and anchor move to
    the projected point at a restart."""
    lp = lpgen.cfg1(1)
    o = OracleOptions(eval_every=1, max_iter=1500, infeas_tol=0.0)
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-30, opts=o, trace_iters=1500)
    restarted = {t: r for t, r, _ in res.log}
    fired = {"suff": 0, "nec": 0, "art": 0}
    last, epoch_R0, prev_R = 0, None, INF
    for t, k, R, R0, R_prev in res.evals:
        assert k == t - last
        if k == 1:
            epoch_R0 = R
        assert R0 == epoch_R0
        assert R_prev == prev_R
        assert restarted[t] == restart_due(R, R0, R_prev, k, t, o)
        if restarted[t]:
            fired["suff" if R <= 0.2 * R0 else "nec" if (R <= 0.8 * R0 and R > R_prev) else "art"] += 1
            x, y, xh, yh = res.trace[t]
            assert np.array_equal(x, xh) and np.array_equal(y, yh)
            last, prev_R = t, INF
        else:
            prev_R = R
    # the run exercises each criterion at least once
    assert all(v > 0 for v in fired.values()), fired


# ---------------------------------------------------------------------------
# initial primal weight
# ---------------------------------------------------------------------------

def test_initial_weight_hand_values():
    assert initial_weight(np.array([3.0, 4.0]), np.array([6.0, 8.0, 0.0])) == 2.0  # ||c~|| / ||b~||
    assert initial_weight(np.array([6.0, 8.0]), np.array([3.0, 0.0, 4.0])) == 0.5
    # the fallback: either norm at or below 1e-10 gives 1
    assert initial_weight(np.zeros(3), np.array([1.0, 2.0])) == 1.0
    assert initial_weight(np.array([1.0, 2.0]), np.zeros(2)) == 1.0
    assert initial_weight(np.array([1e-10]), np.array([5.0])) == 1.0
    assert initial_weight(np.array([5.0]), np.array([1e-10])) == 1.0
    assert initial_weight(np.array([2e-10]), np.array([5.0])) == 5.0 / 2e-10
    assert initial_weight(np.array([5.0]), np.array([2e-10])) == 2e-10 / 5.0


def test_initial_weight_through_the_solve():
    """A = [1 1], b = 2, c = (3, 4).  Ruiz passes leave A alone (every row and
    column maximum is 1); the Pock-Chambolle pass divides the row by sqrt(2)
    (row sum 2) and leaves the columns (sums 1).  So b~ = 2 / sqrt(2) =
    sqrt(2), c~ = (3, 4), omega_0 = 5 / sqrt(2)."""
    A = sp.csr_matrix(np.array([[1.0, 1.0]]))
    res = oracle.solve(A, sp.csr_matrix(A.T), np.array([2.0]), np.array([3.0, 4.0]), 1e-9)
    assert np.allclose(res.d_row, [1.0 / math.sqrt(2.0)], rtol=1e-15)
    assert np.array_equal(res.d_col, [1.0, 1.0])
    assert abs(res.omega0 - 5.0 / math.sqrt(2.0)) <= 1e-15 * 5.0
    assert res.status == 0 and abs(res.meas.pobj - 6.0) <= 1e-8


# ---------------------------------------------------------------------------
# step size: settled and unsettled power iterations
# ---------------------------------------------------------------------------

def _hist(first, last, length=101):
    h = [0.5] * length
    h[-11] = first
    h[-1] = last
    return h


def test_step_size_hand_histories():
    pc, no_pc = OracleOptions(), OracleOptions(pock_chambolle=False)
    # moved by 2^-10 < 1e-3 over the last ten iterations: settled
    h = _hist(1.0 - 2.0 ** -10, 1.0)
    assert step_size(1.0, h, pc) == 0.95
    h = _hist(1.0 - 2.0 ** -10, 0.5)  # sigma_hat is the caller's, not the history's
    assert step_size(0.5, _hist(0.5 - 2.0 ** -11, 0.5), pc) == 0.95 / 0.5
    # moved by 2^-9 > 1e-3: not settled, the safe step
    assert step_size(0.8, _hist(1.0 - 2.0 ** -9, 1.0), pc) == 0.95
    assert step_size(0.8, _hist(1.0 - 2.0 ** -9, 1.0), no_pc) == 0.95 / 0.8
    # exactly 1e-3 relative (1e-3 * 1000 = 1) is settled; a hair more is not
    assert step_size(1000.0, _hist(999.0, 1000.0), pc) == 0.95 / 1000.0
    assert step_size(1000.0, _hist(down(999.0), 1000.0), pc) == 0.95
    # the change is taken against the entry ten iterations back, in either direction
    assert step_size(1000.0, _hist(up(1001.0), 1000.0), pc) == 0.95
    # too short a history to decide, and a zero estimate
    assert step_size(0.8, [0.1, 0.8], pc) == 0.95 / 0.8
    assert step_size(0.0, _hist(0.0, 0.0), pc) == 0.95
    assert step_size(0.8, _hist(1.0 - 2.0 ** -9, 1.0), OracleOptions(step_safety=0.5)) == 0.5


def test_step_size_unsettled_power_iteration():
    lp = lpgen.slow_power_lp(0)
    A = lp.A
    _, _, At = oracle.scale(A)
    s_hat, hist = oracle.power_sigma(At, 100)
    s_max = np.linalg.norm(At.toarray(), 2)
    # dense SVD: the largest singular value is 1 (Pock-Chambolle) and the
    # power estimate is still well below it after 100 iterations
    assert abs(s_max - 1.0) <= 1e-12
    assert s_hat < s_max - 2e-3
    assert abs(hist[-1] - hist[-11]) > 1.5e-3 * hist[-1]
    assert step_size(s_hat, hist, OracleOptions()) == 0.95
    assert step_size(s_hat, hist, OracleOptions(pock_chambolle=False)) == 0.95 / s_hat
    # the solve takes that step, and it is safe: eta * sigma_max < 1
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-9)
    assert res.eta == 0.95 and res.sigma_hat == s_hat
    hi = scipy.optimize.linprog(lp.c, A_eq=A.toarray(), b_eq=lp.b, bounds=(0, None), method="highs")
    assert hi.status == 0 and res.status == 0
    assert abs(res.meas.pobj - hi.fun) <= 1e-7 * (1 + abs(hi.fun))


# ---------------------------------------------------------------------------
# textbook Chambolle-Pock: reflection 0, Halpern off, restarts off
# ---------------------------------------------------------------------------

def _dense_chambolle_pock(A, b, c, tau, sig, iters):
    """x+ = max(x - tau (c - A^T y), 0); y+ = y + sig (b - A (2 x+ - x))."""
    x, y, out = np.zeros(A.shape[1]), np.zeros(A.shape[0]), []
    for _ in range(iters):
        xn = np.maximum(x - tau * (c - A.T @ y), 0.0)
        y = y + sig * (b - A @ (2.0 * xn - x))
        x = xn
        out.append((x, y))
    return out


@pytest.mark.parametrize("lp_fn,scaled", [
    (lambda: lpgen.tiny(5, 12, 3, 0), False),
    (lambda: lpgen.tiny(8, 20, 3, 4), True),
    (lambda: lpgen.cfg1(1), True),
])
def test_textbook_chambolle_pock(lp_fn, scaled):
    lp = lp_fn()
    T = 150
    o = OracleOptions(reflect_rho=0.0, halpern=False, restarts=False, eval_every=10 ** 6,
                      max_iter=T, infeas_tol=0.0)
    if not scaled:
        o.ruiz_iters, o.pock_chambolle = 0, False
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-30, opts=o, trace_iters=T)
    Ad = lp.A.toarray()
    if scaled:
        Ad = res.d_row[:, None] * Ad * res.d_col[None, :]
        bt, ct = res.d_row * lp.b, res.d_col * lp.c
    else:
        assert np.array_equal(res.d_row, np.ones(lp.m)) and np.array_equal(res.d_col, np.ones(lp.n))
        bt, ct = lp.b, lp.c
    tau, sig = res.eta / res.omega0, res.eta * res.omega0
    ref = _dense_chambolle_pock(Ad, bt, ct, tau, sig, T)
    for t in range(1, T + 1):
        x, y, xh, yh = res.trace[t]
        assert np.array_equal(x, xh) and np.array_equal(y, yh)  # no Halpern, no reflection
        rx, ry = ref[t - 1]
        assert np.abs(x - rx).max() <= 1e-12 * max(1.0, np.abs(rx).max())
        assert np.abs(y - ry).max() <= 1e-12 * max(1.0, np.abs(ry).max())
