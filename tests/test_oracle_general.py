"""Pins of the oracle's general form (bounds l <= x <= u, rows of sense
=, >= or <=), handled implicitly by the projections and the evaluation.

Independent references: scipy's HiGHS on the same LP, the planted KKT point
of lpgen (closed-form optimum and a fixed point of the PDHG operator), the
equivalent standard-form LP built here with slack and split variables and
solved by the standard-form oracle, a hand-computed evaluation, and the
special case l = 0, u = +inf, all equalities, which must reproduce the
standard-form run bit for bit.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

import lpgen
import oracle


def _solve_general(lp, eps, **kw):
    return oracle.solve(lp.A, lp.AT, lp.b, lp.c, eps, lo=lp.lo, hi=lp.hi, sense=lp.sense, **kw)


def test_standard_bounds_reproduce_the_standard_run():
    lp = lpgen.cfg1(0)
    a = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-6, trace_iters=100)
    b = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-6, trace_iters=100, lo=np.zeros(lp.n),
                     hi=np.full(lp.n, np.inf), sense=np.zeros(lp.m, dtype=np.int8))
    assert (a.status, a.iters, a.restarts) == (b.status, b.iters, b.restarts)
    for t in range(1, 101):
        for u, v in zip(a.trace[t], b.trace[t]):
            assert np.array_equal(u, v)
    assert np.array_equal(a.meas.x, b.meas.x) and np.array_equal(a.meas.z, b.meas.z)
    assert a.meas.dobj == b.meas.dobj and abs(a.meas.xz - b.meas.xz) <= 1e-12 * (1 + abs(a.meas.xz))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_planted_general_optimum(seed):
    lp = lpgen.general_cfg1(seed)
    # the planted point is feasible and its dual value equals p*
    r = lp.b - lp.A @ lp.x_star
    assert np.abs(r[lp.sense == 0]).max() <= 1e-12
    assert np.all(r[lp.sense == 1] <= 1e-12) and np.all(r[lp.sense == 2] >= -1e-12)
    assert np.all(lp.x_star >= lp.lo) and np.all(lp.x_star <= lp.hi)
    me = oracle.evaluate(lp.A, lp.AT, lp.b, lp.c, np.ones(lp.m), np.ones(lp.n), lp.x_star, lp.y_star,
                         lp.lo, lp.hi, lp.sense)
    assert me.rp_norm <= 1e-12 and me.rd_norm <= 1e-12 and abs(me.dobj - lp.p_star) <= 1e-10
    assert abs(me.xz) <= 1e-12
    res = _solve_general(lp, 1e-8)
    assert res.status == 0
    assert abs(res.meas.pobj - lp.p_star) <= 1e-6 * (1 + abs(lp.p_star))
    # within the bounds up to the rounding of unscaling l / d_c back by d_c
    x = res.meas.x
    tol = 1e-15 * (1 + np.abs(x))
    assert np.all(x >= lp.lo - tol) and np.all(x <= lp.hi + tol)


def test_planted_point_is_a_fixed_point():
    lp = lpgen.general_cfg1(0)
    d_row, d_col, At = oracle.scale(lp.A)
    AtT = sp.csr_matrix(At.T)
    sig_hat, _ = oracle.power_sigma(At)
    eta, omega = 0.95 / sig_hat, 1.7
    tau, sig = eta / omega, eta * omega
    xs, ys = lp.x_star / d_col, lp.y_star / d_row
    xh, yh = oracle.pdhg_operator(At, AtT, d_row * lp.b, d_col * lp.c, tau, sig, xs, ys,
                                  lp.lo / d_col, lp.hi / d_col, lp.sense)
    assert np.abs(xh - xs).max() <= 1e-12 * max(1, np.abs(xs).max())
    assert np.abs(yh - ys).max() <= 1e-12 * max(1, np.abs(ys).max())
    # a wrong sign of one row's projection moves the point off the fixed point
    flip = lp.sense.copy()
    i = int(np.flatnonzero((lp.sense == 1) & (lp.y_star > 0.1))[0])
    flip[i] = 2
    _, yh2 = oracle.pdhg_operator(At, AtT, d_row * lp.b, d_col * lp.c, tau, sig, xs, ys,
                                  lp.lo / d_col, lp.hi / d_col, flip)
    assert abs(yh2[i] - ys[i]) > 1e-3


def _highs(lp):
    A = lp.A.toarray()
    eq, ge, le = lp.sense == 0, lp.sense == 1, lp.sense == 2
    A_ub = np.vstack([-A[ge], A[le]])
    b_ub = np.concatenate([-lp.b[ge], lp.b[le]])
    bounds = [(None if not np.isfinite(l) else l, None if not np.isfinite(u) else u) for l, u in zip(lp.lo, lp.hi)]
    r = linprog(lp.c, A_ub=A_ub if A_ub.size else None, b_ub=b_ub if b_ub.size else None,
                A_eq=A[eq] if eq.any() else None, b_eq=lp.b[eq] if eq.any() else None,
                bounds=bounds, method="highs")
    assert r.status == 0
    return r.fun


@pytest.mark.parametrize("seed", range(4))
def test_general_against_highs(seed):
    lp = lpgen.general_tiny(12, 30, 3, seed)
    f = _highs(lp)
    assert abs(f - lp.p_star) <= 1e-8 * (1 + abs(f))
    res = _solve_general(lp, 1e-9)
    assert res.status == 0
    assert abs(res.meas.pobj - f) <= 1e-6 * (1 + abs(f))


def _to_standard(lp):
    """The same LP in standard form: x = l + x' (x' >= 0) with a row
    x' + s = u - l when u is finite too, x = u - x' with only an upper
    bound, x = x+ - x- when free; a slack per inequality row."""
    A = lp.A.toarray()
    m, n = A.shape
    cols, cost, shift = [], [], np.zeros(n)
    extra_rows = []  # (column index in the new LP, rhs)
    for j in range(n):
        l, u = lp.lo[j], lp.hi[j]
        if np.isfinite(l):
            shift[j] = l
            cols.append(A[:, j])
            cost.append(lp.c[j])
            if np.isfinite(u):
                extra_rows.append((len(cols) - 1, u - l))
        elif np.isfinite(u):
            shift[j] = u
            cols.append(-A[:, j])
            cost.append(-lp.c[j])
        else:
            cols.append(A[:, j])
            cost.append(lp.c[j])
            cols.append(-A[:, j])
            cost.append(-lp.c[j])
    for i in range(m):
        if lp.sense[i] != 0:
            e = np.zeros(m)
            e[i] = -1.0 if lp.sense[i] == 1 else 1.0
            cols.append(e)
            cost.append(0.0)
    N = len(cols)
    top = np.column_stack(cols)
    rows = [top]
    rhs = [lp.b - A @ shift]
    for k, (jc, r) in enumerate(extra_rows):
        row = np.zeros(N + len(extra_rows))
        row[jc] = 1.0
        row[N + k] = 1.0
        rows.append(row[None, :])
        rhs.append(np.array([r]))
    M = np.hstack([rows[0], np.zeros((m, len(extra_rows)))])
    M = np.vstack([M] + rows[1:])
    cst = np.concatenate([cost, np.zeros(len(extra_rows))])
    As = sp.csr_matrix(M)
    return As, sp.csr_matrix(As.T), np.concatenate(rhs), cst, float(lp.c @ shift)


@pytest.mark.parametrize("seed", range(3))
def test_general_against_standard_form_mapping(seed):
    lp = lpgen.general_tiny(10, 24, 3, 100 + seed)
    As, AsT, bs, cs, off = _to_standard(lp)
    ref = oracle.solve(As, AsT, bs, cs, 1e-9)
    res = _solve_general(lp, 1e-9)
    assert ref.status == 0 and res.status == 0
    assert abs((ref.meas.pobj + off) - res.meas.pobj) <= 1e-6 * (1 + abs(res.meas.pobj))


def test_evaluate_by_hand():
    # one row x0 + 2 x1 + x2 + x3 (>= 3 or <= 4); x0 in [0, inf), x1 in
    # [-1, 1], x2 free, x3 in (-inf, 2]; c = 1; at x = (0.5, 1, 0, 2), y = 0.25
    A = sp.csr_matrix(np.array([[1.0, 2.0, 1.0, 1.0]]))
    AT = sp.csr_matrix(A.T)
    lo = np.array([0.0, -1.0, -np.inf, -np.inf])
    hi = np.array([np.inf, 1.0, np.inf, 2.0])
    c = np.ones(4)
    x = np.array([0.5, 1.0, 0.0, 2.0])
    y = np.array([0.25])
    me = oracle.evaluate(A, AT, np.array([3.0]), c, np.ones(1), np.ones(4), x, y, lo, hi,
                         np.array([1], dtype=np.int8))
    # A x = 4.5 >= 3 holds; g = c - A^T y = (0.75, 0.5, 0.75, 0.75)
    assert me.r_p.tolist() == [0.0]
    assert me.z.tolist() == [0.75, 0.5, 0.0, 0.0]
    assert me.r_d.tolist() == [0.0, 0.0, 0.75, 0.75]
    assert me.pobj == 3.5
    assert abs(me.dobj - (0.75 - 0.5)) <= 1e-15       # b y + l1 * 0.5
    assert abs(me.xz - (0.75 * 0.5 + 0.5 * 2.0)) <= 1e-15
    me = oracle.evaluate(A, AT, np.array([4.0]), c, np.ones(1), np.ones(4), x, -y, lo, hi,
                         np.array([2], dtype=np.int8))
    assert me.r_p.tolist() == [-0.5]                  # 4.5 <= 4 is violated by 0.5
    # g = (1.25, 1.5, 1.25, 1.25): lambda = (1.25, 1.5, 0, 0)
    assert me.z.tolist() == [1.25, 1.5, 0.0, 0.0]
    assert abs(me.dobj - (-1.0 - 1.5)) <= 1e-15      # b y + l1 * 1.5


def test_general_validation():
    n, m = 3, 2
    ok = (np.zeros(n), np.ones(n), np.zeros(m, dtype=np.int8))
    oracle.validate_general(n, m, *ok)
    for lo, hi, sense in ((np.ones(n), np.zeros(n), ok[2]), (np.full(n, np.nan), ok[1], ok[2]),
                          (np.full(n, np.inf), np.full(n, np.inf), ok[2]),
                          (ok[0], np.full(n, -np.inf), ok[2]), (ok[0], ok[1], np.full(m, 3, dtype=np.int8))):
        with pytest.raises(ValueError):
            oracle.validate_general(n, m, lo, hi, sense)
