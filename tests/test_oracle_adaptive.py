"""Pins of the adaptive step with rejection (step_rule 1): the rule on
hand-built attempts (accept, reject, the inclusive boundary, a zero or
negative cross term), the bound that makes any step up to 1 / ||A~||_2 safe
(tight for a move along the top singular pair), planted optima reached with
rejections on the way, rejected attempts leaving the iterate unchanged, and
the options the rule needs."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import lpgen
import oracle
from oracle.pdhg import OracleOptions, adaptive_initial_step, adaptive_step, scale

ADAPT = dict(step_rule=1, halpern=False, reflect_rho=0.0)


def test_accepted_attempt_by_hand():
    # omega = 2: (2 * 1 + 4 / 2) / (2 * 1) = 2 >= 0.5; next step
    # min((1 - 2^-0.3) * 2, (1 + 2^-0.6) * 0.5) = min(0.375495..., 0.829877...)
    ok, nxt, bar = adaptive_step(1.0, 4.0, 1.0, 0.5, 2.0, 1)
    assert ok and bar == 2.0
    assert nxt == pytest.approx(0.37549520728752894, rel=1e-15)


def test_rejected_attempt_by_hand():
    ok, nxt, bar = adaptive_step(1.0, 4.0, 1.0, 3.0, 2.0, 1)
    assert not ok and bar == 2.0
    assert nxt == pytest.approx(0.37549520728752894, rel=1e-15)
    # a small eta_bar bound loses to the growth bound when eta is small
    ok, nxt, _ = adaptive_step(1.0, 4.0, 1.0, 0.1, 2.0, 1)
    assert ok and nxt == pytest.approx(0.1 * 1.6597539553864471, rel=1e-15)


def test_boundary_is_accepted_and_the_cross_term_counts_by_magnitude():
    ok, _, bar = adaptive_step(1.0, 1.0, 0.5, 2.0, 1.0, 5)  # eta_bar = 2 / 1 = 2 exactly
    assert bar == 2.0 and ok
    assert not adaptive_step(1.0, 1.0, 0.5, math.nextafter(2.0, 3.0), 1.0, 5)[0]
    assert adaptive_step(1.0, 4.0, -1.0, 0.5, 2.0, 1)[:2] == adaptive_step(1.0, 4.0, 1.0, 0.5, 2.0, 1)[:2]


def test_zero_cross_term_accepts_and_grows_the_step():
    ok, nxt, bar = adaptive_step(1.0, 1.0, 0.0, 1.5, 1.0, 3)
    assert ok and math.isinf(bar)
    assert nxt == pytest.approx(1.5 * 1.4352752816480621, rel=1e-15)  # (1 + 4^-0.6) eta


def test_steps_up_to_the_inverse_norm_are_never_rejected():
    # |dy^T A dx| <= ||A||_2 ||dx|| ||dy|| <= ||A||_2 (omega ||dx||^2 + ||dy||^2 / omega) / 2
    rng = np.random.default_rng(0)
    for trial in range(200):
        m, n = rng.integers(2, 9, size=2)
        A = rng.standard_normal((m, n))
        nrm = np.linalg.norm(A, 2)
        dx, dy = rng.standard_normal(n), rng.standard_normal(m)
        omega = float(np.exp(rng.uniform(-3, 3)))
        ok, _, bar = adaptive_step(dx @ dx, dy @ dy, dy @ A @ dx, 1.0 / nrm, omega, trial + 1)
        assert ok and bar >= (1.0 - 1e-12) / nrm


def test_the_bound_is_tight_along_the_top_singular_pair():
    # dx = a v1, dy = b u1 with omega a^2 = b^2 / omega: eta_bar = 1 / sigma_1
    rng = np.random.default_rng(1)
    A = rng.standard_normal((5, 7))
    U, S, Vt = np.linalg.svd(A)
    omega = 3.0
    a = 0.7
    b = a * omega
    dx, dy = a * Vt[0], b * U[:, 0]
    _, _, bar = adaptive_step(dx @ dx, dy @ dy, dy @ A @ dx, 1.0, omega, 1)
    assert bar == pytest.approx(1.0 / S[0], rel=1e-12)
    assert adaptive_step(dx @ dx, dy @ dy, dy @ A @ dx, (1 - 1e-9) / S[0], omega, 1)[0]
    assert not adaptive_step(dx @ dx, dy @ dy, dy @ A @ dx, (1 + 1e-9) / S[0], omega, 1)[0]


def test_initial_step_is_the_inverse_largest_scaled_entry():
    lp = lpgen.tiny(6, 14, 3, 2)
    _, _, At = scale(lp.A)
    assert adaptive_initial_step(At) == 1.0 / np.abs(At.toarray()).max()
    assert adaptive_initial_step(sp.csr_matrix((2, 3))) == 1.0


@pytest.mark.parametrize("make", [lambda: lpgen.tiny(40, 120, 40, 0), lambda: lpgen.tiny(12, 30, 12, 3),
                                  lambda: lpgen.cfg1(0)])
def test_reaches_the_planted_optimum(make):
    lp = make()
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-8, opts=OracleOptions(**ADAPT))
    assert res.status == 0
    assert abs(res.meas.pobj - lp.p_star) <= 1e-6 * (1 + abs(lp.p_star))
    assert res.sigma_hat == 0.0  # no power iteration


def test_rejections_leave_the_iterate_and_reach_both_parities():
    # the 40 x 120 dense LP rejects its first attempt; the 12 x 30 one rejects
    # attempts 1025 and 1026, right after a restart changed omega
    for lp, T, expect in ((lpgen.tiny(40, 120, 40, 0), 40, [1]), (lpgen.tiny(12, 30, 12, 3), 1100, [1025, 1026])):
        res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-12, opts=OracleOptions(max_iter=T, **ADAPT), trace_iters=T)
        same = []
        prev = (np.zeros(lp.n), np.zeros(lp.m))
        for t in range(1, T + 1):
            x, y, xe, ye = res.trace[t]
            if np.array_equal(x, prev[0]) and np.array_equal(y, prev[1]):
                same.append(t)
            # the evaluated point of the variant is the iterate itself
            assert np.array_equal(x, xe) and np.array_equal(y, ye)
            prev = (x, y)
        assert same == expect and res.rejected == len(expect)


def test_matches_highs_on_a_general_lp():
    from scipy.optimize import linprog
    lp = lpgen.general_tiny(10, 24, 3, 5)
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-9, opts=OracleOptions(**ADAPT), lo=lp.lo, hi=lp.hi,
                       sense=lp.sense)
    A = lp.A.toarray()
    eq, ge, le = lp.sense == 0, lp.sense == 1, lp.sense == 2
    ref = linprog(lp.c, A_ub=np.vstack([-A[ge], A[le]]), b_ub=np.concatenate([-lp.b[ge], lp.b[le]]),
                  A_eq=A[eq], b_eq=lp.b[eq], bounds=list(zip(lp.lo, np.where(np.isinf(lp.hi), None, lp.hi))),
                  method="highs")
    assert res.status == 0 and ref.status == 0
    assert abs(res.meas.pobj - ref.fun) <= 1e-6 * (1 + abs(ref.fun))


@pytest.mark.parametrize("bad", [dict(halpern=True), dict(reflect_rho=1.0), dict(restart_avg=True)])
def test_needs_plain_pdhg(bad):
    lp = lpgen.tiny(6, 14, 3, 0)
    with pytest.raises(ValueError):
        oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-6, opts=OracleOptions(**dict(ADAPT, **bad)))


def test_off_is_the_default_run():
    lp = lpgen.cfg1(1)
    a = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-8)
    b = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-8, opts=OracleOptions(step_rule=0))
    assert (a.iters, a.restarts, a.rejected) == (b.iters, b.restarts, 0) and np.array_equal(a.meas.x, b.meas.x)
