"""GPU interior-point consumer against the oracle's (oracle/ipm.py): cold
starts (Newton steps, first step lengths, the optimum), warm starts from a
PDHG solution through Algorithm 1 (steps and the alpha_min loop), the loop's
lifts on a start that touches the boundary, the hybrid end to end, and the
inputs it refuses."""
import numpy as np
import pytest
import scipy.sparse as sp

import lpgen
import oracle
from oracle import ipm as I
from oracle.pdhg import scale

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_03150_amd")
torch = pytest.importorskip("torch")


def _np(t):
    return t.detach().cpu().numpy()


def _dev(v):
    return torch.as_tensor(np.ascontiguousarray(v), dtype=torch.float64, device="cuda")


def _scaled(lp):
    d_row, d_col, _ = scale(lp.A)
    At, bt, ct = I.scaled_lp(lp.A, lp.b, lp.c, d_row, d_col)
    return At, bt, ct, d_row, d_col


@pytest.mark.parametrize("make", [lambda: lpgen.tiny(30, 90, 3, 1), lambda: lpgen.cfg1(0),
                                  lambda: lpgen.tiny(40, 120, 40, 0), lambda: lpgen.cfg2_sub(0, 100)])
def test_cold_start_matches_oracle(make):
    lp = make()
    At, bt, ct, d_row, d_col = _scaled(lp)
    ref = I.ipm(At, bt, ct)
    sol = P.ipm_solve(P.DeviceLP.from_lp(lp), _dev(d_row), _dev(d_col))
    info = sol.info
    assert sol.status == ref.status == 0
    assert info["iters"] == ref.iters
    assert info["first_step_p"] == pytest.approx(ref.steps[0][0], rel=1e-9)
    assert info["first_step_d"] == pytest.approx(ref.steps[0][1], rel=1e-9)
    assert info["pivots_replaced"] == 0
    assert abs(info["pobj"] - lp.p_star) <= 1e-7 * (1 + abs(lp.p_star))
    # the same point (the method's limit is the analytic centre of the optimal face)
    assert np.linalg.norm(_np(sol.x) / d_col - ref.x) <= 1e-6 * (1 + np.linalg.norm(ref.x))
    assert np.linalg.norm(_np(sol.y) / d_row - ref.y) <= 1e-6 * (1 + np.linalg.norm(ref.y))


def test_unscaled_solve():
    lp = lpgen.tiny(20, 50, 6, 3)
    ones_r, ones_c = np.ones(lp.m), np.ones(lp.n)
    At, bt, ct = I.scaled_lp(lp.A, lp.b, lp.c, ones_r, ones_c)
    ref = I.ipm(At, bt, ct)
    sol = P.ipm_solve(P.DeviceLP.from_lp(lp))
    assert sol.status == 0 and sol.info["iters"] == ref.iters
    assert abs(sol.info["pobj"] - lp.p_star) <= 1e-7 * (1 + abs(lp.p_star))


@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_warm_start_from_the_oracles_pdhg_solution(eps):
    lp = lpgen.cfg2_sub(0, 100)
    At, bt, ct, d_row, d_col = _scaled(lp)
    pd = oracle.solve(lp.A, lp.AT, lp.b, lp.c, eps)
    m = pd.meas
    ref = I.warm_ipm(At, bt, ct, m.x / d_col, m.y / d_row, m.z * d_col)
    sol = P.ipm_warm(P.DeviceLP.from_lp(lp), _PdhgPoint(m.x, m.y, m.z, d_row, d_col))
    info = sol.info
    assert sol.status == ref.ipm.status == 0
    assert (info["iters"], info["lifts"]) == (ref.ipm.iters, ref.lifts)
    assert info["mu_target"] == pytest.approx(ref.mu_target, rel=1e-12)
    assert info["first_step_p"] == pytest.approx(ref.ipm.steps[0][0], rel=1e-8)
    assert abs(info["pobj"] - lp.p_star) <= 1e-7 * (1 + abs(lp.p_star))


class _PdhgPoint:
    """A PDHG solution in the original space with its scaling, as ipm_warm takes it."""

    def __init__(self, x, y, z, d_row, d_col):
        self.x, self.y, self.z, self.d_row, self.d_col = (_dev(v) for v in (x, y, z, d_row, d_col))


@pytest.mark.parametrize("make,kw,lifts", [
    # centring off (delta_max 0) from the 1e-4 PDHG point: first steps 2e-8, 2e-7, 2e-6 for
    # alpha_min 1e-12, 1e-11, 1e-10, so the paper's minimum step 1e-6 takes two lifts
    (lambda: lpgen.cfg1(0), dict(mu_min=1e-14, delta_max=0.0, alpha_min=1e-12, min_step=1e-6), 2),
    # first steps 0.008, 0.009, 0.02, 0.94 for alpha_min 1e-10 .. 1e-7
    (lambda: lpgen.tiny(30, 90, 3, 1), dict(mu_min=1e-14, delta_max=0.0, alpha_min=1e-10, min_step=0.5), 3),
    # no first step reaches 0.99999 (step_frac 0.9995 caps it): max_lifts lifts
    (lambda: lpgen.tiny(30, 90, 3, 1), dict(alpha_min=1e-10, min_step=0.99999, max_lifts=4), 4),
])
def test_recovery_loop_lifts_like_the_oracle(make, kw, lifts):
    lp = make()
    At, bt, ct, d_row, d_col = _scaled(lp)
    m = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-4).meas
    ref = I.warm_ipm(At, bt, ct, m.x / d_col, m.y / d_row, m.z * d_col, **kw)
    assert ref.lifts == lifts
    sol = P.ipm_warm(P.DeviceLP.from_lp(lp), _PdhgPoint(m.x, m.y, m.z, d_row, d_col), **kw)
    assert sol.info["lifts"] == lifts and sol.info["alpha_min"] == pytest.approx(ref.alpha_min, rel=1e-12)
    assert sol.info["iters"] == ref.ipm.iters and sol.status == ref.ipm.status


def test_hybrid_end_to_end_takes_fewer_iterations():
    # the GPU PDHG to 1e-4, Algorithm 1, the GPU interior-point method; against its cold start
    for lp in (lpgen.cfg1(0), lpgen.cfg2_sub(0, 100)):
        dlp = P.DeviceLP.from_lp(lp)
        pd = P.solve(dlp, 1e-4, "fp64")
        warm = P.ipm_warm(dlp, pd)
        cold = P.ipm_solve(dlp, pd.d_row, pd.d_col)
        assert warm.status == cold.status == 0
        assert warm.info["iters"] < cold.info["iters"] and warm.info["iters"] <= 10
        assert abs(warm.info["pobj"] - lp.p_star) <= 1e-7 * (1 + abs(lp.p_star))


def test_refused_inputs():
    with pytest.raises(P.MipdhgError) as e:
        P.ipm_solve(P.DeviceLP.from_lp(lpgen.general_tiny(10, 24, 3, 5)))
    assert e.value.code == -6
    lp = lpgen.tiny(6, 14, 3, 0)
    dlp = P.DeviceLP.from_lp(lp)
    with pytest.raises(P.MipdhgError) as e:
        P.ipm_solve(dlp, start=(torch.ones(lp.n, dtype=torch.float64, device="cuda"), None, None))
    assert e.value.code == -1
    with pytest.raises(P.MipdhgError) as e:
        P.ipm_solve(dlp, tol=0.0)
    assert e.value.code == -1
    # a row whose columns are out of order
    A = lp.A.copy()
    r = int(np.argmax(np.diff(A.indptr) >= 2))
    s, t = A.indptr[r], A.indptr[r + 1]
    A.indices[s:t] = A.indices[s:t][::-1].copy()
    A.data[s:t] = A.data[s:t][::-1].copy()
    bad = P.DeviceLP(A, sp.csr_matrix(A.toarray().T), lp.b, lp.c, "cuda")
    with pytest.raises(P.MipdhgError) as e:
        P.ipm_solve(bad)
    assert e.value.code == -2
