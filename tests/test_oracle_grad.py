"""Pins of the oracle's reverse mode for the unrolled PDHG map x_K(c, b).

With the restart schedule and the steps frozen, the map is piecewise linear in
(c, b); away from projection-mask flips a central finite difference is exact up
to rounding, so it checks the adjoint without using it.  A forward-mode
(tangent) pass gives a second, independent derivation: <J v, w> = <v, J^T w>.
"""
import numpy as np
import pytest

import lpgen
import oracle
from oracle.pdhg import OracleOptions

K_FD = 300


def _fd_check(lp, w, K, h=1e-6, ncomp=12, seed=0):
    opts = OracleOptions()
    gc, gb, xK, sched = oracle.unrolled_grad(lp.A, lp.b, lp.c, K, w, opts)
    _, _, tape0 = oracle.unrolled_forward(lp.A, lp.b, lp.c, K, opts, sched, keep_masks=True)
    masks0 = np.array(tape0["masks"])
    rng = np.random.default_rng(seed)
    checked = skipped = 0
    for which, g, size in (("c", gc, lp.n), ("b", gb, lp.m)):
        for j in rng.choice(size, size=min(ncomp, size), replace=False):
            e = np.zeros(size)
            e[j] = h
            if which == "c":
                xp, _, tp = oracle.unrolled_forward(lp.A, lp.b, lp.c + e, K, opts, sched, keep_masks=True)
                xm, _, tm = oracle.unrolled_forward(lp.A, lp.b, lp.c - e, K, opts, sched, keep_masks=True)
            else:
                xp, _, tp = oracle.unrolled_forward(lp.A, lp.b + e, lp.c, K, opts, sched, keep_masks=True)
                xm, _, tm = oracle.unrolled_forward(lp.A, lp.b - e, lp.c, K, opts, sched, keep_masks=True)
            if not (np.array_equal(np.array(tp["masks"]), masks0)
                    and np.array_equal(np.array(tm["masks"]), masks0)):
                skipped += 1
                continue
            fd = (w @ xp - w @ xm) / (2 * h)
            assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j])) + 1e-8, (which, j, fd, g[j])
            checked += 1
    return checked, skipped


@pytest.mark.parametrize("inst", [0, 1, 2])
def test_fd_small_instances(inst):
    lp, w = lpgen.cfg5_fd_instance(inst)
    checked, skipped = _fd_check(lp, w, K_FD, seed=inst)
    assert checked >= 16, (checked, skipped)


def test_dot_product_reverse_vs_tangent():
    lp, w = lpgen.cfg5_fd_instance(5)
    opts = OracleOptions()
    K = 200
    gc, gb, xK, sched = oracle.unrolled_grad(lp.A, lp.b, lp.c, K, w, opts)
    rng = np.random.default_rng(9)
    for _ in range(3):
        dc = rng.normal(size=lp.n)
        db = rng.normal(size=lp.m)
        dx, _, _ = oracle.unrolled_tangent(lp.A, lp.b, lp.c, K, dc, db, opts, sched)
        lhs = float(w @ dx)
        rhs = float(gc @ dc + gb @ db)
        assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))


def test_schedule_replay_is_identity():
    lp, w = lpgen.cfg5_fd_instance(3)
    x1, sched, _ = oracle.unrolled_forward(lp.A, lp.b, lp.c, 400)
    x2, _, _ = oracle.unrolled_forward(lp.A, lp.b, lp.c, 400, schedule=sched)
    assert np.array_equal(x1, x2)
    assert len(sched.restart_at) >= 1 and len(sched.taus) == len(sched.restart_at) + 1


def test_unrolled_matches_solve_trajectory():
    # with no termination inside K iterations, the unrolled map follows the
    # same iterates as the solve loop
    lp = lpgen.cfg1(0)
    K = 150
    xK, sched, _ = oracle.unrolled_forward(lp.A, lp.b, lp.c, K)
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-30,
                       opts=OracleOptions(max_iter=K), trace_iters=K)
    xh = res.trace[K][2]
    assert np.allclose(xK, res.d_col * xh, rtol=1e-13, atol=1e-13)
    assert [t for t, r, _ in res.log if r] == sched.restart_at
