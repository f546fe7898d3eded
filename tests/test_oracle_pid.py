"""Pins of the PID primal-weight variant: with a constant distance ratio r the
controller's fixed point is omega = r (with an integral gain its sum settles
at zero); gains (theta, 0, 0) are the smoothing rule; a hand-computed first
and second update; a PID run still converges to the planted optimum."""
import math

import pytest

import lpgen
import oracle
from oracle.pdhg import OracleOptions


@pytest.mark.parametrize("ki,kd", [(0.1, 0.0), (0.1, 0.2), (0.0, 0.3), (0.05, 0.1)])
def test_controller_settles_at_the_ratio(ki, kd):
    opts = OracleOptions(pw_theta=0.5, pw_ki=ki, pw_kd=kd)
    pid = [0.0, 0.0, 0]
    omega, dx, dy = 1.0, 2.0, 7.4  # r = 3.7
    for _ in range(400):
        omega = oracle.primal_weight_update(omega, dx, dy, pid, opts)
    assert abs(omega - 3.7) <= 1e-9 * 3.7
    if ki > 0:
        assert abs(pid[0]) <= 1e-9  # with an integral gain its sum returns to zero


def test_zero_gains_are_the_smoothing_rule():
    opts = OracleOptions(pw_theta=0.3)
    pid = [0.0, 0.0, 0]
    w = oracle.primal_weight_update(2.0, 1.5, 4.0, pid, opts)
    assert w == math.exp(0.3 * math.log(4.0 / 1.5) + 0.7 * math.log(2.0)) and pid == [0.0, 0.0, 0]


def test_first_update_by_hand():
    # e = log(2) - log(4/1) = -log 2; I = e; no derivative at the first update
    opts = OracleOptions(pw_theta=0.5, pw_ki=0.1, pw_kd=0.7)
    pid = [0.0, 0.0, 0]
    w = oracle.primal_weight_update(2.0, 1.0, 4.0, pid, opts)
    e = -math.log(2.0)
    assert abs(w - math.exp(math.log(2.0) - (0.5 * e + 0.1 * e))) <= 1e-15
    # second update at the same ratio: derivative e2 - e
    w2 = oracle.primal_weight_update(w, 1.0, 4.0, pid, opts)
    e2 = math.log(w) - math.log(4.0)
    assert abs(w2 - math.exp(math.log(w) - (0.5 * e2 + 0.1 * (e + e2) + 0.7 * (e2 - e)))) <= 1e-14


def test_pid_run_reaches_the_planted_optimum():
    lp = lpgen.cfg1(0)
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-8, opts=OracleOptions(pw_ki=0.1, pw_kd=0.2))
    assert res.status == 0 and res.restarts > 0
    assert abs(res.meas.pobj - lp.p_star) <= 1e-6 * (1 + abs(lp.p_star))
