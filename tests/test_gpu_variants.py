"""GPU parity of the method variants against the oracle: the PID primal
weight (per-iterate FP64 parity across restarts, full-solve iteration and
restart counts), and its refusal by the batched and unrolled solves."""
import numpy as np
import pytest

import lpgen
import oracle
from oracle.pdhg import OracleOptions

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_03150_amd")
torch = pytest.importorskip("torch")


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b)) / max(1.0, float(np.linalg.norm(b)))


@pytest.mark.parametrize("ki,kd", [(0.1, 0.3), (0.02, 0.0)])
def test_pid_trace_parity(ki, kd):
    lp = lpgen.cfg2_sub(0, 100)
    T = 320
    sol = P.solve(P.DeviceLP.from_lp(lp), 1e-12, "fp64", trace_iters=T, max_iter=T, eval_every=16, pw_ki=ki,
                  pw_kd=kd)
    ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-12, opts=OracleOptions(max_iter=T, eval_every=16, pw_ki=ki,
                                                                           pw_kd=kd), trace_iters=T)
    assert ref.restarts >= 3 and sol.info["restarts"] == ref.restarts
    assert abs(sol.info["omega"] - ref.omega) <= 1e-9 * ref.omega
    for t in range(1, T + 1):
        xs, ys, xh, yh = ref.trace[t]
        for key, r in (("x", xs), ("y", ys), ("xhat", xh), ("yhat", yh)):
            assert _rel(_np(sol.trace[key][t - 1]), r) <= 1e-9, (t, key)


def test_pid_full_solve_matches_oracle():
    lp = lpgen.cfg1(0)
    kw = dict(pw_ki=0.1, pw_kd=0.2)
    sol = P.solve(P.DeviceLP.from_lp(lp), 1e-8, "fp64", **kw)
    ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-8, opts=OracleOptions(**kw))
    assert sol.status == ref.status == 0
    assert sol.info["iters"] == ref.iters and sol.info["restarts"] == ref.restarts
    assert _rel(_np(sol.x), ref.meas.x) <= 1e-8


def test_pid_is_a_single_lp_option():
    batch = P.DeviceBatch.from_lps([lpgen.tiny(6, 15, 3, 0)])
    with pytest.raises(P.MipdhgError) as e:
        P.solve_batched(batch, 1e-4, "fp32", pw_ki=0.1)
    assert e.value.code == -6


@pytest.mark.parametrize("kw", [dict(), dict(gather_order=1), dict(tile_nnz=4096, tile_nnz_at=512, tile_rows_at=64)])
def test_restart_to_average_trace_parity(kw):
    lp = lpgen.cfg2_sub(1, 100)
    T = 320
    opts = dict(halpern=0, restart_avg=1, eval_every=16)
    sol = P.solve(P.DeviceLP.from_lp(lp), 1e-12, "fp64", trace_iters=T, max_iter=T, **opts, **kw)
    ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-12, trace_iters=T,
                       opts=OracleOptions(max_iter=T, eval_every=16, halpern=False, restart_avg=True))
    assert ref.restarts >= 3 and sol.info["restarts"] == ref.restarts
    for t in range(1, T + 1):
        xs, ys, xh, yh = ref.trace[t]
        for key, r in (("x", xs), ("y", ys), ("xhat", xh), ("yhat", yh)):
            assert _rel(_np(sol.trace[key][t - 1]), r) <= 1e-9, (t, key)


@pytest.mark.parametrize("halpern", [0, 1])
def test_restart_to_average_full_solve(halpern):
    lp = lpgen.cfg1(2)
    sol = P.solve(P.DeviceLP.from_lp(lp), 1e-7, "fp64", halpern=halpern, restart_avg=1)
    ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-7, opts=OracleOptions(halpern=bool(halpern), restart_avg=True))
    assert sol.status == ref.status == 0
    assert sol.info["iters"] == ref.iters and sol.info["restarts"] == ref.restarts
    # float32 iterates reach the tolerance too
    s32 = P.solve(P.DeviceLP.from_lp(lp), 1e-4, "fp32", halpern=halpern, restart_avg=1)
    assert s32.status == 0


def test_restart_to_average_limits():
    lp = lpgen.cfg1(0)
    with pytest.raises(P.MipdhgError) as e:
        P.solve(P.DeviceLP.from_lp(lp), 1e-4, "fp64", restart_avg=1, spmv_kind=2)
    assert e.value.code == -6
    batch = P.DeviceBatch.from_lps([lpgen.tiny(6, 15, 3, 0)])
    with pytest.raises(P.MipdhgError) as e:
        P.solve_batched(batch, 1e-4, "fp32", restart_avg=1)
    assert e.value.code == -6
    best = P.autotune(P.DeviceLP.from_lp(lp), "fp64", iters=16, restart_avg=1)
    assert best["spmv_kind"] == 0


@pytest.mark.parametrize("kw", [dict(), dict(halpern=0, restart_avg=1), dict(restart_avg=1), dict(spmv_kind=3)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_workspace_contents_do_not_matter(kw, prec):
    # a workspace full of NaN bit patterns gives bitwise the solve of a zeroed one:
    # nothing is read before the solve writes it (the epoch average included)
    dlp = P.DeviceLP.from_lp(lpgen.cfg2_sub(0, 100))
    nb = P.workspace_bytes(dlp, prec, **kw)
    zero = torch.zeros(nb, dtype=torch.uint8, device=dlp.device)
    junk = torch.full((nb,), 0xFF, dtype=torch.uint8, device=dlp.device)
    a = P.solve(dlp, 1e-6, prec, workspace=zero, max_iter=2000, **kw)
    b = P.solve(dlp, 1e-6, prec, workspace=junk, max_iter=2000, **kw)
    assert a.status == b.status and a.status != 3
    assert a.info["iters"] == b.info["iters"] and torch.equal(a.x, b.x) and torch.equal(a.y, b.y)
