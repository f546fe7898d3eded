"""GPU infeasibility certificates against the oracle's: the same status at
the same iteration (FP64) on infeasible and unbounded LPs in both forms, the
status in FP32 (certificate tolerance 1e-5), and no certificate test when
infeas_tol = 0."""
import pytest

import lpgen
import oracle
from oracle.pdhg import OracleOptions

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_03150_amd")
torch = pytest.importorskip("torch")

CASES = [lpgen.farkas_tiny, lpgen.unbounded_tiny, lpgen.box_infeasible, lambda: lpgen.conflicting_rows(0),
         lambda: lpgen.conflicting_rows(1), lambda: lpgen.unbounded_column(0), lambda: lpgen.unbounded_column(1)]


def _kw(lp):
    return dict(lo=lp.lo, hi=lp.hi, sense=lp.sense) if lp.general else {}


@pytest.mark.parametrize("make", CASES)
@pytest.mark.parametrize("spmv_kind", [0, 2])
def test_certificate_matches_oracle_fp64(make, spmv_kind):
    lp = make()
    ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-6, opts=OracleOptions(max_iter=20_000), **_kw(lp))
    assert ref.status in (4, 5)
    sol = P.solve(P.DeviceLP.from_lp(lp), 1e-6, "fp64", max_iter=20_000, spmv_kind=spmv_kind)
    assert sol.status == ref.status and sol.info["iters"] == ref.iters, (sol.status_name, sol.info["iters"], ref.iters)


@pytest.mark.parametrize("make", CASES)
def test_certificate_fp32(make):
    # float32 iterates carry ~6e-8 relative rounding that grows with the
    # drifting iterate, so the certificate tolerance is 1e-5 there
    lp = make()
    ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-6, opts=OracleOptions(max_iter=20_000), **_kw(lp))
    sol = P.solve(P.DeviceLP.from_lp(lp), 1e-6, "fp32", max_iter=20_000, infeas_tol=1e-5)
    assert sol.status == ref.status


def test_tests_off_runs_to_the_limit():
    lp = lpgen.farkas_tiny()
    sol = P.solve(P.DeviceLP.from_lp(lp), 1e-6, "fp64", max_iter=300, infeas_tol=0.0)
    assert sol.status == P.ITER_LIMIT and sol.info["iters"] == 300
    with pytest.raises(P.MipdhgError):
        P.solve(P.DeviceLP.from_lp(lp), 1e-6, "fp64", infeas_tol=-1.0)
