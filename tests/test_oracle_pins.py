"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names what fixes the expected value: a closed form, a brute force,
an independent library solver, a theorem about the PDHG operator, or a
definition from Section 2 / Section 4.3 of the paper.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.optimize
import scipy.sparse as sp

import lpgen
import oracle
from oracle.pdhg import OracleOptions


# ---------------------------------------------------------------------------
# closed form: the planted KKT point fixes the optimal value
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_planted_optimum_cfg1(seed):
    lp = lpgen.cfg1(seed)
    # the planted pair is an exact KKT point (Section 2 optimality conditions)
    assert np.abs(lp.A @ lp.x_star - lp.b).max() < 1e-12
    assert np.abs(lp.AT @ lp.y_star + lp.z_star - lp.c).max() < 1e-12
    assert float(lp.x_star @ lp.z_star) == 0.0
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-8)
    assert res.status == 0
    p_star = lp.p_star
    assert abs(res.meas.pobj - p_star) <= 1e-6 * (1 + abs(p_star))
    assert abs(res.meas.dobj - p_star) <= 1e-6 * (1 + abs(p_star))
    # the point returned satisfies the paper's three tests at 1e-8
    assert res.meas.rp_norm <= 1e-8 * (1 + np.linalg.norm(lp.b))
    assert res.meas.rd_norm <= 1e-8 * (1 + np.linalg.norm(lp.c))
    assert np.all(res.meas.x >= 0) and np.all(res.meas.z >= 0)


def test_planted_optimum_cfg2_sub():
    lp = lpgen.cfg2_sub(0, scale=200)
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-7)
    assert res.status == 0
    assert abs(res.meas.pobj - lp.p_star) <= 1e-5 * (1 + abs(lp.p_star))


# ---------------------------------------------------------------------------
# brute force: vertex enumeration on tiny LPs
# ---------------------------------------------------------------------------

def _vertex_optimum(A: np.ndarray, b: np.ndarray, c: np.ndarray) -> float:
    m, n = A.shape
    best = math.inf
    for basis in itertools.combinations(range(n), m):
        B = A[:, basis]
        if abs(np.linalg.det(B)) < 1e-12:
            continue
        xb = np.linalg.solve(B, b)
        if np.all(xb >= -1e-9):
            best = min(best, float(c[list(basis)] @ xb))
    return best


@pytest.mark.parametrize("m,n,seed", [(3, 7, 0), (4, 9, 1), (5, 10, 2), (5, 12, 3), (6, 12, 4)])
def test_vertex_enumeration(m, n, seed):
    lp = lpgen.tiny(m, n, 3, seed)
    p_v = _vertex_optimum(lp.A.toarray(), lp.b, lp.c)
    assert math.isfinite(p_v)
    assert abs(p_v - lp.p_star) <= 1e-9 * (1 + abs(p_v))
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-10)
    assert res.status == 0
    assert abs(res.meas.pobj - p_v) <= 1e-8 * (1 + abs(p_v))


# ---------------------------------------------------------------------------
# independent library solver: HiGHS through scipy
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 3])
def test_highs_agreement(seed):
    lp = lpgen.cfg1(seed)
    hi = scipy.optimize.linprog(lp.c, A_eq=lp.A, b_eq=lp.b, bounds=(0, None), method="highs")
    assert hi.status == 0
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-9)
    assert abs(res.meas.pobj - hi.fun) <= 1e-7 * (1 + abs(hi.fun))


# ---------------------------------------------------------------------------
# textbook case: m = 1, sum(x) = 1
# ---------------------------------------------------------------------------

def test_simplex_lp():
    c = lpgen.rng_for(77).uniform(-2.0, 3.0, size=9)
    lp = lpgen.simplex_lp(c)
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-10)
    assert res.status == 0
    assert abs(res.meas.pobj - c.min()) <= 1e-8
    assert abs(res.meas.y[0] - c.min()) <= 1e-7
    assert np.allclose(res.meas.z, c - c.min(), atol=1e-7)


# ---------------------------------------------------------------------------
# the PDHG operator: fixed point, firm nonexpansiveness, Halpern rate
# ---------------------------------------------------------------------------

def _scaled_setup(lp, omega=1.0):
    d_row, d_col, At = oracle.scale(lp.A)
    AtT = sp.csr_matrix(At.T)
    sig_hat, hist = oracle.power_sigma(At)
    eta = 0.95 / sig_hat
    return d_row, d_col, At, AtT, eta / omega, eta * omega


def test_operator_fixed_point():
    lp = lpgen.cfg1(0)
    d_row, d_col, At, AtT, tau, sig = _scaled_setup(lp, omega=2.0)
    xs = lp.x_star / d_col
    ys = lp.y_star / d_row
    xh, yh = oracle.pdhg_operator(At, AtT, d_row * lp.b, d_col * lp.c, tau, sig, xs, ys)
    assert np.abs(xh - xs).max() <= 1e-12 * max(1, np.abs(xs).max())
    assert np.abs(yh - ys).max() <= 1e-12 * max(1, np.abs(ys).max())
    # started at the planted point, the solve stops at its first evaluation
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-10, x_init=lp.x_star, y_init=lp.y_star)
    assert res.status == 0 and res.iters == 64


def _M_inner(At, tau, sig, dx, dy, ex, ey):
    """<(dx,dy),(ex,ey)>_M with M = [[I/tau, At^T], [At, I/sig]], the metric in
    which the PDHG operator is firmly nonexpansive (for tau*sig*||At||^2 < 1)."""
    return dx @ ex / tau + dy @ ey / sig + dy @ (At @ ex) + ey @ (At @ dx)


def test_operator_firmly_nonexpansive():
    lp = lpgen.tiny(8, 20, 3, 5)
    d_row, d_col, At, AtT, tau, sig = _scaled_setup(lp, omega=1.7)
    bt, ct = d_row * lp.b, d_col * lp.c
    rng = np.random.default_rng(1)
    for _ in range(500):
        x1, x2 = rng.normal(size=(2, 20))
        y1, y2 = rng.normal(size=(2, 8))
        a1, b1 = oracle.pdhg_operator(At, AtT, bt, ct, tau, sig, x1, y1)
        a2, b2 = oracle.pdhg_operator(At, AtT, bt, ct, tau, sig, x2, y2)
        lhs = _M_inner(At, tau, sig, a1 - a2, b1 - b2, a1 - a2, b1 - b2)
        rhs = _M_inner(At, tau, sig, a1 - a2, b1 - b2, x1 - x2, y1 - y2)
        assert lhs <= rhs + 1e-10 * max(1.0, abs(rhs))


@pytest.mark.parametrize("rho", [1.0, 0.5])
def test_halpern_residual_bound(rho):
    """Halpern iteration on the nonexpansive S = (1+rho) T - rho I with weights
    (k+1)/(k+2) obeys ||z_k - S z_k|| <= 2 ||z_0 - z*|| / (k+1) (Lieder 2021),
    i.e. ||z_k - T z_k||_M <= 2 ||z_0 - z*||_M / ((1+rho)(k+1))."""
    lp = lpgen.tiny(10, 25, 3, 7)
    opts = OracleOptions(restarts=False, reflect_rho=rho, eval_every=10_000, max_iter=400)
    res = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-30, opts=opts, trace_iters=400)
    d_row, d_col, At = oracle.scale(lp.A)
    tau, sig = res.eta / res.omega0, res.eta * res.omega0
    xs, ys = lp.x_star / d_col, lp.y_star / d_row
    r0 = math.sqrt(_M_inner(At, tau, sig, xs, ys, xs, ys))  # z_0 = 0
    prev = (np.zeros(25), np.zeros(10))
    for t in range(1, 401):
        xk, yk, xh, yh = res.trace[t]
        # trace[t] holds T(z_{t-1}) = (xh, yh); z_{t-1} = prev
        dx, dy = prev[0] - xh, prev[1] - yh
        fp = math.sqrt(max(0.0, _M_inner(At, tau, sig, dx, dy, dx, dy)))
        assert fp <= 2.0 * r0 / ((1.0 + rho) * t) * (1 + 1e-9) + 1e-13
        prev = (xk, yk)


# ---------------------------------------------------------------------------
# evaluation: definitions of Section 2 and Section 4.3
# ---------------------------------------------------------------------------

def test_kkt_gap_identity():
    lp = lpgen.cfg1(1)
    rng = np.random.default_rng(3)
    d_row = rng.uniform(0.5, 2.0, lp.m)
    d_col = rng.uniform(0.5, 2.0, lp.n)
    xh = np.maximum(rng.normal(size=lp.n), 0)
    yh = rng.normal(size=lp.m)
    me = oracle.evaluate(lp.A, lp.AT, lp.b, lp.c, d_row, d_col, xh, yh)
    lhs = me.pobj - me.dobj
    rhs = me.x @ me.z + me.x @ me.r_d - me.y @ me.r_p
    assert abs(lhs - rhs) <= 1e-10 * (1 + abs(lhs))
    assert np.all(me.z >= 0)
    assert np.allclose(me.x, d_col * xh) and np.allclose(me.y, d_row * yh)


def test_evaluate_known_residual():
    lp = lpgen.cfg1(2)
    j = int(np.flatnonzero(lp.x_star > 0)[0])
    delta = 1e-3
    x = lp.x_star.copy()
    x[j] += delta
    me = oracle.evaluate(lp.A, lp.AT, lp.b, lp.c, np.ones(lp.m), np.ones(lp.n), x, lp.y_star)
    col = lp.A[:, j].toarray().ravel()
    assert np.allclose(me.r_p, -delta * col, atol=1e-13)
    assert me.rd_norm <= 1e-12
    assert abs(me.gap - delta * abs(lp.z_star[j] + lp.AT[j] @ lp.y_star)) <= 1e-12 * (1 + me.gap)
    # maximum violation (Section 4.3)
    assert me.violation == max(me.rp_inf, me.rd_inf, me.xz / (1 + abs(me.pobj)))


def test_termination_just_pass_just_fail():
    lp = lpgen.cfg1(0)
    nb, nc = np.linalg.norm(lp.b), np.linalg.norm(lp.c)
    eps = 1e-4
    base = oracle.evaluate(lp.A, lp.AT, lp.b, lp.c, np.ones(lp.m), np.ones(lp.n),
                           lp.x_star, lp.y_star)
    assert oracle.terminated(base, nb, nc, eps)

    def with_(**kw):
        d = dict(base.__dict__)
        d.update(kw)
        return oracle.Measures(**d)

    thr_p = eps * (1 + nb)
    thr_d = eps * (1 + nc)
    assert oracle.terminated(with_(rp_norm=thr_p), nb, nc, eps)  # inclusive
    assert not oracle.terminated(with_(rp_norm=thr_p * (1 + 1e-12)), nb, nc, eps)
    assert oracle.terminated(with_(rd_norm=thr_d), nb, nc, eps)
    assert not oracle.terminated(with_(rd_norm=thr_d * (1 + 1e-12)), nb, nc, eps)
    p, d = base.pobj, base.dobj
    thr_g = eps * (1 + abs(p) + abs(d))
    assert oracle.terminated(with_(gap=thr_g), nb, nc, eps)
    assert not oracle.terminated(with_(gap=thr_g * (1 + 1e-12)), nb, nc, eps)


# ---------------------------------------------------------------------------
# scaling and step size
# ---------------------------------------------------------------------------

def test_scaling_definition_and_invariants():
    lp = lpgen.cfg2_sub(0, scale=200)
    d_row, d_col, At = oracle.scale(lp.A, ruiz_iters=10, pock_chambolle=True)
    ref = sp.diags(d_row) @ lp.A @ sp.diags(d_col)
    assert abs(ref - At).max() <= 1e-13 * abs(At).max()
    assert np.all(d_row > 0) and np.all(d_col > 0)
    # Pock-Chambolle (alpha = 1) bounds the spectral norm by 1 (Schur test)
    s_max = np.linalg.norm(At.toarray(), 2)
    assert s_max <= 1 + 1e-12
    # many Ruiz passes equilibrate infinity norms of non-empty rows/columns
    d_row2, d_col2, At2 = oracle.scale(lp.A, ruiz_iters=40, pock_chambolle=False)
    a = abs(At2)
    rmax = np.asarray(a.max(axis=1).todense()).ravel()
    cmax = np.asarray(a.max(axis=0).todense()).ravel()
    assert np.all(np.abs(rmax[rmax > 0] - 1) < 1e-3)
    assert np.all(np.abs(cmax[cmax > 0] - 1) < 1e-3)


def test_power_iteration_diagonal_closed_form():
    # diag(a): the power iteration on diag(a^2) from 1/sqrt(n) converges to max|a|
    a = np.array([0.3, -0.9, 0.5, 0.7, -0.2, 0.6])
    s_hat, hist = oracle.power_sigma(sp.csr_matrix(np.diag(a)), 100)
    assert abs(s_hat - 0.9) <= 1e-12
    # first estimate is ||diag(a) 1/sqrt(n)|| = ||a|| / sqrt(n)
    assert abs(hist[0] - np.linalg.norm(a) / math.sqrt(a.size)) <= 1e-15


def test_scaling_closed_forms():
    rng = np.random.default_rng(11)
    # a scaled permutation: one Ruiz pass (and one Pock-Chambolle pass) make
    # every entry +-1
    n = 7
    perm = rng.permutation(n)
    vals = rng.uniform(0.1, 10, n) * rng.choice([-1, 1], n)
    P = sp.csr_matrix((vals, (np.arange(n), perm)), shape=(n, n))
    for ruiz, pc in ((1, False), (0, True)):
        d_row, d_col, At = oracle.scale(P, ruiz, pc)
        assert np.allclose(np.abs(At.data), 1.0, rtol=0, atol=1e-15)
        assert np.allclose(d_row * d_col[perm], 1.0 / np.abs(vals), rtol=1e-15)
    # |A| = u v^T (rank one, positive): one Ruiz pass gives
    # sqrt(u_i v_j) / sqrt(max u max v); one Pock-Chambolle pass gives
    # sqrt(u_i v_j) / sqrt(sum u sum v)
    u = rng.uniform(0.5, 4, 5)
    v = rng.uniform(0.5, 4, 8)
    sgn = rng.choice([-1.0, 1.0], (5, 8))
    R1 = sp.csr_matrix(sgn * np.outer(u, v))
    _, _, At = oracle.scale(R1, 1, False)
    assert np.allclose(np.abs(At.toarray()), np.sqrt(np.outer(u, v)) / math.sqrt(u.max() * v.max()),
                       rtol=1e-14)
    _, _, At = oracle.scale(R1, 0, True)
    assert np.allclose(np.abs(At.toarray()), np.sqrt(np.outer(u, v)) / math.sqrt(u.sum() * v.sum()),
                       rtol=1e-14)


@pytest.mark.parametrize("seed", [0, 1])
def test_power_iteration_vs_dense_norm(seed):
    lp = lpgen.cfg1(seed)
    _, _, At = oracle.scale(lp.A)
    s_hat, hist = oracle.power_sigma(At, 100)
    s_max = np.linalg.norm(At.toarray(), 2)
    assert s_hat <= s_max * (1 + 1e-12)
    assert s_hat >= 0.998 * s_max
    # the Rayleigh estimates never decrease
    assert all(hist[i + 1] >= hist[i] * (1 - 1e-12) for i in range(len(hist) - 1))


def test_empty_row_and_validation():
    # an empty row (b_i = 0) is allowed; its scale factor is 1 and y_i stays 0
    A = sp.csr_matrix(np.array([[1.0, 1.0, 0.0], [0.0, 0.0, 0.0]]))
    lp_b = np.array([1.0, 0.0])
    c = np.array([1.0, 2.0, 0.5])
    AT = sp.csr_matrix(A.T)
    res = oracle.solve(A, AT, lp_b, c, 1e-9)
    assert res.status == 0 and res.d_row[1] == 1.0
    assert abs(res.meas.pobj - 1.0) < 1e-7 and res.meas.y[1] == 0.0
    with pytest.raises(ValueError):
        oracle.solve(A, sp.csr_matrix(A.T * 2), lp_b, c, 1e-4)
    with pytest.raises(ValueError):
        oracle.solve(A, AT, np.array([np.nan, 0.0]), c, 1e-4)


def test_iteration_limit_and_infeasible():
    # x1 + x2 = -1 with x >= 0 is infeasible: without the certificate tests
    # no termination (ITER_LIMIT); with them, primal infeasibility at the
    # second evaluation
    A = sp.csr_matrix(np.array([[1.0, 1.0]]))
    res = oracle.solve(A, sp.csr_matrix(A.T), np.array([-1.0]), np.array([1.0, 1.0]), 1e-6,
                       opts=OracleOptions(max_iter=300, infeas_tol=0.0))
    assert res.status == 1 and res.iters == 300
    assert res.meas.rp_norm > 0.5
    res = oracle.solve(A, sp.csr_matrix(A.T), np.array([-1.0]), np.array([1.0, 1.0]), 1e-6,
                       opts=OracleOptions(max_iter=300))
    assert res.status == 4 and res.iters == 128
