"""Pins of the oracle's infeasibility certificates: scipy's HiGHS classifies
the same LPs (infeasible: status 2, unbounded: status 3), hand-checked
certificate quantities, and no certificate on solvable planted LPs (their
runs are the same with the tests on and off)."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

import lpgen
import oracle
from oracle.pdhg import OracleOptions


def _highs_status(A, b, c, lo=None, hi=None, sense=None):
    A = np.asarray(A.toarray() if sp.issparse(A) else A, dtype=float)
    m, n = A.shape
    lo = np.zeros(n) if lo is None else lo
    hi = np.full(n, np.inf) if hi is None else hi
    sense = np.zeros(m, dtype=np.int8) if sense is None else sense
    eq, ge, le = sense == 0, sense == 1, sense == 2
    A_ub = np.vstack([-A[ge], A[le]])
    b_ub = np.concatenate([-b[ge], b[le]])
    bounds = [(None if not np.isfinite(l) else l, None if not np.isfinite(u) else u) for l, u in zip(lo, hi)]
    r = linprog(c, A_ub=A_ub if A_ub.size else None, b_ub=b_ub if b_ub.size else None,
                A_eq=A[eq] if eq.any() else None, b_eq=b[eq] if eq.any() else None, bounds=bounds,
                method="highs")
    return r.status


def _solve(A, b, c, **kw):
    A = sp.csr_matrix(A)
    return oracle.solve(A, sp.csr_matrix(A.T), b, c, 1e-6, opts=OracleOptions(max_iter=20_000), **kw)


def test_farkas_ray_by_hand():
    # x1 + x2 = -1, x >= 0: e = -1 gives A^T e = (-1, -1) <= 0 and b^T e = 1 > 0
    A = sp.csr_matrix(np.array([[1.0, 1.0]]))
    q_e, r_e, q_d, r_d = oracle.ray_measures(A, sp.csr_matrix(A.T), np.array([-1.0]), np.ones(2),
                                             np.zeros(2), np.array([-1.0]))
    assert (q_e, r_e) == (1.0, 0.0)
    assert oracle.infeasibility(q_e, r_e, q_d, r_d, 1e-8) == 4
    # e = +1 is not a certificate: its value is negative
    q_e, r_e, _, _ = oracle.ray_measures(A, sp.csr_matrix(A.T), np.array([-1.0]), np.ones(2),
                                         np.zeros(2), np.array([1.0]))
    assert q_e < 0 and oracle.infeasibility(q_e, r_e, 0.0, 0.0, 1e-8) is None


def test_primal_ray_by_hand():
    # min -x1 s.t. x1 - x2 = 0, x >= 0: d = (1, 1) has A d = 0, d >= 0, c^T d = -1
    A = sp.csr_matrix(np.array([[1.0, -1.0]]))
    q_e, r_e, q_d, r_d = oracle.ray_measures(A, sp.csr_matrix(A.T), np.zeros(1), np.array([-1.0, 0.0]),
                                             np.array([1.0, 1.0]), np.zeros(1))
    assert (q_d, r_d) == (-1.0, 0.0)
    assert oracle.infeasibility(q_e, r_e, q_d, r_d, 1e-8) == 5
    # with x2 <= 3 the direction leaves the bounds' recession cone
    lo, hi = np.zeros(2), np.array([np.inf, 3.0])
    _, _, q_d, r_d = oracle.ray_measures(A, sp.csr_matrix(A.T), np.zeros(1), np.array([-1.0, 0.0]),
                                         np.array([1.0, 1.0]), np.zeros(1), lo, hi, np.zeros(1, dtype=np.int8))
    assert r_d == 1.0 and oracle.infeasibility(0.0, 0.0, q_d, r_d, 1e-8) is None


def test_standard_form_infeasible_and_unbounded():
    A = np.array([[1.0, 1.0]])
    b, c = np.array([-1.0]), np.array([1.0, 1.0])
    assert _highs_status(A, b, c) == 2
    assert _solve(A, b, c).status == 4
    A = np.array([[1.0, -1.0]])
    b, c = np.array([0.0]), np.array([-1.0, 0.0])
    assert _highs_status(A, b, c) == 3
    assert _solve(A, b, c).status == 5


@pytest.mark.parametrize("make,highs,want", [
    (lambda: lpgen.conflicting_rows(0), 2, 4), (lambda: lpgen.conflicting_rows(1), 2, 4),
    (lambda: lpgen.unbounded_column(0), 3, 5), (lambda: lpgen.unbounded_column(1), 3, 5),
    (lpgen.box_infeasible, 2, 4), (lpgen.farkas_tiny, 2, 4), (lpgen.unbounded_tiny, 3, 5)])
def test_lps_without_optimum_against_highs(make, highs, want):
    lp = make()
    assert _highs_status(lp.A, lp.b, lp.c, lp.lo, lp.hi, lp.sense) == highs
    kw = dict(lo=lp.lo, hi=lp.hi, sense=lp.sense) if lp.general else {}
    res = _solve(lp.A, lp.b, lp.c, **kw)
    assert res.status == want


@pytest.mark.parametrize("make", [lambda: lpgen.cfg1(0), lambda: lpgen.cfg1(3), lambda: lpgen.general_cfg1(0),
                                  lambda: lpgen.general_cfg1(2), lambda: lpgen.cfg2_sub(0, 100)])
def test_no_certificate_on_solvable_lps(make):
    lp = make()
    kw = dict(lo=lp.lo, hi=lp.hi, sense=lp.sense) if lp.general else {}
    a = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-8, **kw)
    b = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-8, opts=OracleOptions(infeas_tol=0.0), **kw)
    assert a.status == b.status == 0 and a.iters == b.iters
