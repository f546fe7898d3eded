"""Pins of the restart-to-average variant: the restart point is the plain
mean of the epoch's projected points (checked against numpy's mean of the
traced points), the option off leaves the run unchanged, and runs with it
reach the planted optimum."""
import numpy as np
import pytest

import lpgen
import oracle
from oracle.pdhg import OracleOptions


def test_restart_point_is_the_epoch_mean():
    lp = lpgen.cfg1(0)
    T = 640
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-12, trace_iters=T,
                       opts=OracleOptions(halpern=False, restart_avg=True, max_iter=T))
    restarts = [t for t, r, _ in res.log if r]
    assert len(restarts) >= 2
    start = 1
    for t in restarts:
        xs = np.array([res.trace[s][2] for s in range(start, t + 1)])
        ys = np.array([res.trace[s][3] for s in range(start, t + 1)])
        # after a restart the state is the restart point
        assert np.allclose(res.trace[t][0], xs.mean(axis=0), rtol=1e-12, atol=1e-14)
        assert np.allclose(res.trace[t][1], ys.mean(axis=0), rtol=1e-12, atol=1e-14)
        start = t + 1


def test_option_off_is_the_default_run():
    lp = lpgen.cfg1(1)
    a = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-8)
    b = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-8, opts=OracleOptions(restart_avg=False))
    assert (a.iters, a.restarts) == (b.iters, b.restarts) and np.array_equal(a.meas.x, b.meas.x)


@pytest.mark.parametrize("halpern", [False, True])
def test_restart_to_average_reaches_the_planted_optimum(halpern):
    lp = lpgen.cfg1(2)
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-7, opts=OracleOptions(halpern=halpern, restart_avg=True))
    assert res.status == 0 and res.restarts > 0
    assert abs(res.meas.pobj - lp.p_star) <= 1e-5 * (1 + abs(lp.p_star))
