"""Checkpoint/resume of the single-LP solve: a solve stopped at an evaluation
and resumed from its workspace gives bitwise the iterates, iteration count and
restart count of one uninterrupted solve, and a workspace that holds another
problem's (or another layout's) state is refused."""
import pytest

import lpgen

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_03150_amd")
torch = pytest.importorskip("torch")


def _same(a, b):
    assert a.status == b.status
    assert a.info["iters"] == b.info["iters"] and a.info["restarts"] == b.info["restarts"]
    for k in ("x", "y", "z", "r_p", "r_d"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    assert a.info["omega"] == b.info["omega"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("spmv_kind", [0, 2])
def test_resume_at_iteration_limit_matches_one_solve(prec, spmv_kind):
    dlp = P.DeviceLP.from_lp(lpgen.cfg2_sub(6, scale=100))
    kw = dict(spmv_kind=spmv_kind)
    ref = P.solve(dlp, 1e-12, prec, max_iter=320, **kw)
    assert ref.status == 1 and ref.info["restarts"] > 0
    a = P.solve(dlp, 1e-12, prec, max_iter=128, **kw)
    assert a.status == 1 and a.info["iters"] == 128
    b = P.solve(dlp, 1e-12, prec, max_iter=192, resume=a, **kw)
    assert b.info["iters"] == 192
    c = P.solve(dlp, 1e-12, prec, max_iter=320, resume=b, **kw)
    _same(ref, c)


def test_resume_direct_launches_and_graph_agree():
    dlp = P.DeviceLP.from_lp(lpgen.cfg1(2))
    ref = P.solve(dlp, 1e-12, "fp64", max_iter=256, use_graph=1)
    a = P.solve(dlp, 1e-12, "fp64", max_iter=64, use_graph=0)
    b = P.solve(dlp, 1e-12, "fp64", max_iter=256, use_graph=1, resume=a)
    _same(ref, b)


def test_resume_after_optimal_with_tighter_tolerance():
    dlp = P.DeviceLP.from_lp(lpgen.cfg2_sub(6, scale=100))
    ref = P.solve(dlp, 1e-7, "fp64")
    loose = P.solve(dlp, 1e-3, "fp64")
    assert loose.status == 0 and loose.info["iters"] < ref.info["iters"]
    tight = P.solve(dlp, 1e-7, "fp64", resume=loose)
    _same(ref, tight)


def test_resume_of_an_optimal_state_stops_at_once():
    dlp = P.DeviceLP.from_lp(lpgen.cfg1(1))
    a = P.solve(dlp, 1e-6, "fp64")
    assert a.status == 0
    x = a.x.clone()
    it = a.info["iters"]
    b = P.solve(dlp, 1e-6, "fp64", max_iter=10 * it, resume=a)
    assert b.status == 0 and b.info["iters"] == it and torch.equal(b.x, x)


def test_resume_refuses_another_state():
    lp = lpgen.cfg1(1)
    dlp = P.DeviceLP.from_lp(lp)
    a = P.solve(dlp, 1e-12, "fp64", max_iter=64)
    # other options that shape the state or its layout
    for kw in (dict(precision="fp32"), dict(eval_every=32), dict(tile_nnz=512), dict(gather_order=1)):
        prec = kw.pop("precision", "fp64")
        with pytest.raises((P.MipdhgError, ValueError)):
            P.solve(dlp, 1e-12, prec, max_iter=128, resume=a, **kw)
    # the same sizes but another right-hand side
    other = P.DeviceLP.from_lp(lp)
    other.b.mul_(1.5)
    with pytest.raises(P.MipdhgError) as e:
        P.solve(other, 1e-12, "fp64", max_iter=128, resume=a)
    assert e.value.code == -1
    # a refused resume leaves the state usable
    ref = P.solve(dlp, 1e-12, "fp64", max_iter=128)
    b = P.solve(dlp, 1e-12, "fp64", max_iter=128, resume=a)
    _same(ref, b)
    # back-to-back kernel timing moves the iterates: not resumable
    t = P.solve(dlp, 1e-12, "fp64", max_iter=64, kernel_timing=2)
    with pytest.raises(P.MipdhgError) as e:
        P.solve(dlp, 1e-12, "fp64", max_iter=128, resume=t)
    assert e.value.code == -1
    # a workspace never used by a solve
    fresh = P.solve(dlp, 1e-12, "fp64", max_iter=64)
    fresh.workspace.zero_()
    with pytest.raises(P.MipdhgError):
        P.solve(dlp, 1e-12, "fp64", max_iter=128, resume=fresh)
    # no warm start with a resume
    with pytest.raises(P.MipdhgError):
        P.solve(dlp, 1e-12, "fp64", max_iter=128, resume=a, x_init=torch.zeros(lp.n))


def test_resume_is_refused_by_the_unrolled_map():
    # the batched solve resumes its blocks (test_gpu_batched.py); the unrolled
    # map has no state to continue
    batch = P.DeviceBatch.from_lps([lpgen.tiny(6, 15, 3, 0)])
    with pytest.raises(P.MipdhgError) as e:
        P.UnrolledMap(batch, K=8, ckpt_every=4, precision="fp32", resume=1)
    assert e.value.code == -6
    with pytest.raises(TypeError):
        P.solve_batched(batch, 1e-4, "fp32", resume=1)


def test_time_limit_stops_at_a_block_and_resumes_bitwise():
    # a limit that has passed once the first block is queued: the solve stops
    # after that block (TIME_LIMIT), and resuming it is one uninterrupted solve
    dlp = P.DeviceLP.from_lp(lpgen.cfg2_sub(6, scale=100))
    ref = P.solve(dlp, 1e-7, "fp64")
    a = P.solve(dlp, 1e-7, "fp64", time_limit_s=1e-9)
    assert a.status == P.TIME_LIMIT and a.info["iters"] == 64
    b = P.solve(dlp, 1e-7, "fp64", resume=a)
    _same(ref, b)


def test_resume_general_form():
    lp = lpgen.general_cfg1(1)
    dlp = P.DeviceLP.from_lp(lp)
    ref = P.solve(dlp, 1e-12, "fp64", max_iter=256)
    a = P.solve(dlp, 1e-12, "fp64", max_iter=128)
    b = P.solve(dlp, 1e-12, "fp64", max_iter=256, resume=a)
    _same(ref, b)
    # the same matrix and data as a standard-form LP is another state
    std = P.DeviceLP(lp.A, lp.AT, lp.b, lp.c)
    c = P.solve(dlp, 1e-12, "fp64", max_iter=64)
    with pytest.raises(P.MipdhgError):
        P.solve(std, 1e-12, "fp64", max_iter=128, resume=c)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_exported_state_resumes_in_a_new_workspace(prec):
    dlp = P.DeviceLP.from_lp(lpgen.cfg2_sub(6, scale=100))
    ref = P.solve(dlp, 1e-12, prec, max_iter=320)
    a = P.solve(dlp, 1e-12, prec, max_iter=128)
    state = P.export_state(dlp, a, prec)
    assert state.device.type == "cpu" and state.numel() == P.state_bytes(dlp, prec)
    a.workspace.zero_()  # the original workspace is gone
    ws = P.import_state(dlp, state, prec)
    b = P.solve(dlp, 1e-12, prec, max_iter=320, resume=ws)
    _same(ref, b)
    # a state of other options does not import into this layout's checks
    with pytest.raises(P.MipdhgError):
        P.import_state(dlp, state[:-8], prec)


@pytest.mark.parametrize("kw", [dict(halpern=0, restart_avg=1), dict(pw_ki=0.1, pw_kd=0.2)])
def test_variant_states_export_and_resume(kw):
    # the epoch averages and the PID state travel with the exported state
    lp = lpgen.general_cfg1(2)
    dlp = P.DeviceLP.from_lp(lp)
    ref = P.solve(dlp, 1e-12, "fp64", max_iter=384, eval_every=32, **kw)
    assert ref.info["restarts"] >= 2
    a = P.solve(dlp, 1e-12, "fp64", max_iter=160, eval_every=32, **kw)
    ws = P.import_state(dlp, P.export_state(dlp, a, "fp64", eval_every=32, **kw), "fp64", eval_every=32, **kw)
    b = P.solve(dlp, 1e-12, "fp64", max_iter=384, eval_every=32, resume=ws, **kw)
    _same(ref, b)
