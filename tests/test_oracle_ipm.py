"""Pins of the interior-point consumer (oracle/ipm.py): optima of planted LPs
and scipy's HiGHS, the Newton direction against the linearised KKT system
that defines it, Mehrotra's start against numpy's minimum-norm least squares,
hand-built ratio tests and centering parameters, warm starts from a
perturbed optimum, and the alpha_min recovery loop."""
import numpy as np
import pytest

import lpgen
from oracle import ipm as I
from oracle.pdhg import scale


def _scaled(lp):
    d_row, d_col, _ = scale(lp.A)
    At, bt, ct = I.scaled_lp(lp.A, lp.b, lp.c, d_row, d_col)
    return At, bt, ct, d_row, d_col


@pytest.mark.parametrize("make", [lambda: lpgen.cfg1(0), lambda: lpgen.tiny(30, 90, 3, 1),
                                  lambda: lpgen.tiny(40, 120, 40, 0)])
def test_cold_start_reaches_the_planted_optimum(make):
    lp = make()
    At, bt, ct, d_row, d_col = _scaled(lp)
    r = I.ipm(At, bt, ct)
    assert r.status == 0 and max(r.rel) <= 1e-8
    # c~^T x~ = c^T x: the objective is scale-free
    assert abs(float(ct @ r.x) - lp.p_star) <= 1e-7 * (1 + abs(lp.p_star))
    assert 3 <= r.iters <= 40 and np.all(r.x > 0) and np.all(r.z > 0)


def test_matches_highs():
    from scipy.optimize import linprog
    lp = lpgen.tiny(20, 50, 6, 3)
    At, bt, ct, _, _ = _scaled(lp)
    r = I.ipm(At, bt, ct)
    ref = linprog(lp.c, A_eq=lp.A.toarray(), b_eq=lp.b, bounds=(0, None), method="highs")
    assert r.status == 0 and ref.status == 0
    assert abs(float(ct @ r.x) - ref.fun) <= 1e-7 * (1 + abs(ref.fun))


def test_newton_direction_solves_the_linearised_kkt_system():
    lp = lpgen.tiny(15, 40, 4, 0)
    At, bt, ct, _, _ = _scaled(lp)
    rng = np.random.default_rng(1)
    x, z = rng.uniform(0.1, 2.0, lp.n), rng.uniform(0.1, 2.0, lp.n)
    y = rng.standard_normal(lp.m)
    r_b, r_c = bt - At @ x, ct - At.T @ y - z
    r_xz = rng.standard_normal(lp.n)
    dx, dy, dz = I.newton(At, x, z, r_b, r_c, r_xz)
    assert np.allclose(At @ dx, r_b, rtol=0, atol=1e-10)
    assert np.allclose(At.T @ dy + dz, r_c, rtol=0, atol=1e-10)
    assert np.allclose(z * dx + x * dz, r_xz, rtol=0, atol=1e-10)


def test_mehrotra_start_is_the_shifted_least_squares_point():
    lp = lpgen.tiny(15, 40, 4, 2)
    At, bt, ct, _, _ = _scaled(lp)
    x0, y0, z0 = I.mehrotra_start(At, bt, ct)
    Ad = At.toarray()
    x_ls = np.linalg.lstsq(Ad, bt, rcond=None)[0]  # minimum norm for full row rank
    y_ls = np.linalg.lstsq(Ad.T, ct, rcond=None)[0]
    assert np.allclose(y0, y_ls, atol=1e-10)
    sx, sz = x0 - x_ls, z0 - (ct - Ad.T @ y_ls)
    assert np.ptp(sx) <= 1e-10 and np.ptp(sz) <= 1e-10  # each a constant shift
    assert np.all(x0 > 0) and np.all(z0 > 0)


def test_ratio_test_and_centering_parameter_by_hand():
    assert I.boundary_step(np.array([1.0, 2.0, 3.0]), np.array([-1.0, 1.0, -6.0])) == 0.5
    assert I.boundary_step(np.array([1.0, 2.0]), np.array([0.0, 3.0])) == np.inf
    assert I.centering_sigma(0.5, 2.0) == 1.0 / 64.0


def test_warm_start_from_a_perturbed_optimum_takes_few_iterations():
    lp = lpgen.cfg1(2)
    At, bt, ct, d_row, d_col = _scaled(lp)
    rng = np.random.default_rng(3)
    x = lp.x_star / d_col + 1e-5 * rng.uniform(0, 1, lp.n)
    z = lp.z_star * d_col + 1e-5 * rng.uniform(0, 1, lp.n)
    y = lp.y_star / d_row + 1e-5 * rng.standard_normal(lp.m)
    h = I.warm_ipm(At, bt, ct, x, y, z)
    cold = I.ipm(At, bt, ct)
    assert h.ipm.status == 0 and h.lifts == 0
    assert h.ipm.iters <= 5 < cold.iters
    assert abs(float(ct @ h.ipm.x) - lp.p_star) <= 1e-7 * (1 + abs(lp.p_star))


def test_recovery_loop_lifts_alpha_min():
    lp = lpgen.tiny(12, 30, 4, 2)
    At, bt, ct, d_row, d_col = _scaled(lp)
    xs, zs = lp.x_star / d_col, lp.z_star * d_col
    y = lp.y_star / d_row + 1e-3 * np.random.default_rng(0).standard_normal(lp.m)
    kw = dict(mu_min=1e-14, delta_max=1e-14, alpha_min=1e-12)
    # no first step reaches 0.99999 (eta = 0.9995 caps it): alpha_min grows max_lifts times
    h = I.warm_ipm(At, bt, ct, xs, y, zs, min_step=0.99999, max_lifts=4, **kw)
    assert h.lifts == 4 and h.alpha_min == pytest.approx(1e-8, rel=1e-12)
    # from 1e-12 the first step is 0.999486; after one lift (1e-11) it is 0.999499
    h = I.warm_ipm(At, bt, ct, xs, y, zs, min_step=0.99949, **kw)
    assert h.lifts == 1 and h.alpha_min == pytest.approx(1e-11, rel=1e-12)
    assert min(h.ipm.steps[0]) >= 0.99949 and h.ipm.status == 0
