"""GPU parity of the batched persistent solve against the float64 oracle.

FP64: every instance matches the oracle run on that instance alone: status,
iteration count, restart count, and the returned point (over thousands of
iterations rounding-order differences grow, so the point is compared at the
solve tolerance; the first 150 iterations are compared at 1e-10).  FP32: every
instance satisfies the Section 2 tests when re-measured in float64 on the
host, and its objective obeys the bound the planted KKT pair implies.
"""
import numpy as np
import pytest
import scipy.sparse as sp

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


def _sizes(count, lo=20, hi=300, seed=0):
    rng = lpgen.rng_for(44, seed)
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))).astype(int)


def objective_bound(lp, x, y):
    """|c^T x - p*| <= ||y*|| ||r_P|| + ||x*|| ||r_D|| + |c^T x - b^T y| for
    the planted optimum: c^T x - p* = z*^T x - y*^T r_P >= -||y*|| ||r_P||, and
    p* - b^T y = z^T x* + r_D^T x* >= -||x*|| ||r_D|| with z = max(c - A^T y, 0)."""
    z = np.maximum(lp.c - lp.AT @ y, 0.0)
    rp = lp.b - lp.A @ x
    rd = lp.c - lp.AT @ y - z
    gap = abs(lp.c @ x - lp.b @ y)
    bound = np.linalg.norm(lp.y_star) * np.linalg.norm(rp) + np.linalg.norm(lp.x_star) * np.linalg.norm(rd) + gap
    return abs(lp.c @ x - lp.p_star), bound


def _tests_hold(lp, x, y, eps):
    z = np.maximum(lp.c - lp.AT @ y, 0.0)
    rp = lp.b - lp.A @ x
    rd = lp.c - lp.AT @ y - z
    p, d = lp.c @ x, lp.b @ y
    return (np.linalg.norm(rp) <= eps * (1 + np.linalg.norm(lp.b))
            and np.linalg.norm(rd) <= eps * (1 + np.linalg.norm(lp.c))
            and abs(p - d) <= eps * (1 + abs(p) + abs(d)))


@pytest.mark.parametrize("split", [0, 2048])
def test_batched_fp64_matches_oracle_per_instance(split):
    # split 2048: instances with m + n > 254 run in the wide workgroups
    lps = [lpgen.cfg4_instance(i, m) for i, m in enumerate(_sizes(24))]
    batch = P.DeviceBatch.from_lps(lps)
    eps = 1e-6
    sol = P.solve_batched(batch, eps, "fp64", max_iter=100_000, batch_split=split)
    for i, lp in enumerate(lps):
        ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, eps, opts=OracleOptions(max_iter=100_000))
        got = sol.split(batch, i)
        assert got["info"]["status"] == ref.status == 0, i
        assert got["info"]["iters"] == ref.iters, (i, got["info"]["iters"], ref.iters)
        assert got["info"]["restarts"] == ref.restarts, i
        assert _rel(_np(got["x"]), ref.meas.x) <= eps, i
        assert _rel(_np(got["y"]), ref.meas.y) <= eps, i
        assert abs(got["info"]["sigma_hat"] - ref.sigma_hat) <= 1e-12 * ref.sigma_hat
        assert np.linalg.norm(_np(got["r_p"]) - ref.meas.r_p) <= eps * (1 + np.linalg.norm(lp.b))


def test_batched_fp64_iteration_limit_and_options():
    # a tail evaluation at max_iter, no Halpern, no restarts, rho = 0.5
    lps = [lpgen.cfg4_instance(100 + i, m) for i, m in enumerate([20, 37, 64])]
    batch = P.DeviceBatch.from_lps(lps)
    kw = dict(max_iter=150, halpern=0, restarts=0, reflect_rho=0.5)
    sol = P.solve_batched(batch, 1e-12, "fp64", **kw)
    for i, lp in enumerate(lps):
        ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-12,
                           opts=OracleOptions(max_iter=150, halpern=False, restarts=False, reflect_rho=0.5))
        got = sol.split(batch, i)
        assert got["info"]["status"] == ref.status == 1 and got["info"]["iters"] == 150
        assert _rel(_np(got["x"]), ref.meas.x) <= 1e-10


@pytest.mark.parametrize("split", [0, 4096])
@pytest.mark.parametrize("T", [1, 64, 100, 257])
def test_batched_fp64_iterates_match_oracle_at_default_options(T, split):
    """Per-iterate parity with the default options (Halpern, reflection 1,
    restarts): cut at iteration T by the iteration limit, every instance's
    evaluated point equals the oracle's after T iterations, on sizes up to
    m = 2,000 (LDS-resident instances of every size the batch holds); with
    split 4096 the three larger instances run in the wide workgroups."""
    sizes = [20, 150, 700, 2000]
    lps = [lpgen.cfg4_instance(600 + i, m) for i, m in enumerate(sizes)]
    batch = P.DeviceBatch.from_lps(lps)
    sol = P.solve_batched(batch, 1e-14, "fp64", max_iter=T, batch_split=split)
    for i, lp in enumerate(lps):
        ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-14, opts=OracleOptions(max_iter=T))
        got = sol.split(batch, i)
        assert got["info"]["status"] == ref.status == 1 and got["info"]["iters"] == T
        assert got["info"]["restarts"] == ref.restarts, i
        assert _rel(_np(got["x"]), ref.meas.x) <= 1e-10, (i, T)
        assert _rel(_np(got["y"]), ref.meas.y) <= 1e-10, (i, T)


def test_batched_fp32_reaches_tolerance():
    lps = [lpgen.cfg4_instance(200 + i, m) for i, m in enumerate(_sizes(64, 20, 2000, seed=1))]
    batch = P.DeviceBatch.from_lps(lps)
    eps = 1e-4
    sol = P.solve_batched(batch, eps, "fp32", max_iter=200_000)
    assert sol.status == 0
    for i in range(0, len(lps), 7):
        lp = lps[i]
        got = sol.split(batch, i)
        x, y = _np(got["x"]), _np(got["y"])
        assert _tests_hold(lp, x, y, eps), i
        err, bound = objective_bound(lp, x, y)
        assert err <= bound * (1 + 1e-9) + 1e-12, (i, err, bound)


def test_batched_single_instance_equals_plain_solve():
    lp = lpgen.cfg1(0)
    b = P.solve_batched(P.DeviceBatch.from_lps([lp]), 1e-6, "fp64")
    p = P.solve(P.DeviceLP.from_lp(lp), 1e-6, "fp64")
    assert b.infos[0]["iters"] == p.info["iters"]
    assert _rel(_np(b.x), _np(p.x)) <= 1e-10


def test_batched_deterministic():
    lps = [lpgen.cfg4_instance(300 + i, m) for i, m in enumerate(_sizes(40, seed=2))]
    batch = P.DeviceBatch.from_lps(lps)
    a = P.solve_batched(batch, 1e-4, "fp32")
    b = P.solve_batched(batch, 1e-4, "fp32")
    assert torch.equal(a.x, b.x) and torch.equal(a.y, b.y)
    assert [i["iters"] for i in a.infos] == [i["iters"] for i in b.infos]


def test_batched_rejects_off_block_entry():
    lps = [lpgen.cfg4_instance(400 + i, 30) for i in range(2)]
    batch = P.DeviceBatch.from_lps(lps)
    # move one entry of instance 0 into instance 1's columns
    batch.lp.a_col[0] = int(batch.col_off[1]) + 1
    with pytest.raises(P.MipdhgError) as e:
        P.solve_batched(batch, 1e-4, "fp64")
    assert e.value.code in (-2, -3)


def test_batched_rejects_consistent_off_block_pair():
    """Off-block entries with A^T the exact transpose: only the block check
    can see them."""
    ob = lpgen.off_block_pair()
    batch = P.DeviceBatch(ob.A, ob.AT, ob.b, ob.c, ob.row_off, ob.col_off, ob.nnz_off, device="cuda")
    with pytest.raises(P.MipdhgError) as e:
        P.solve_batched(batch, 1e-4, "fp64")
    assert e.value.code == -2 and "outside" in str(e.value)


def test_batched_per_instance_tolerances():
    """Each instance stops by its own eps_rel (Section 2 tests): the same LP
    twice at 1e-3 and 1e-7 takes the iterations the single-LP solve takes at
    each tolerance, and each returned point passes its own tests."""
    lp = lpgen.cfg1(2)
    eps = [1e-3, 1e-7]
    b = P.solve_batched(P.DeviceBatch.from_lps([lp, lp]), eps, "fp64")
    nb, nc = np.linalg.norm(lp.b), np.linalg.norm(lp.c)
    its = []
    for i, e in enumerate(eps):
        p = P.solve(P.DeviceLP.from_lp(lp), e, "fp64")
        assert b.infos[i]["status"] == 0 and b.infos[i]["iters"] == p.info["iters"], (i, e)
        its.append(b.infos[i]["iters"])
        x = _np(b.x)[lp.n * i:lp.n * (i + 1)]
        y = _np(b.y)[lp.m * i:lp.m * (i + 1)]
        rp = lp.b - lp.A @ x
        rd = lp.c - lp.AT @ y - np.maximum(lp.c - lp.AT @ y, 0.0)
        pv, dv = lp.c @ x, lp.b @ y
        assert np.linalg.norm(rp) <= e * (1 + nb) and np.linalg.norm(rd) <= e * (1 + nc)
        assert abs(pv - dv) <= e * (1 + abs(pv) + abs(dv))
    assert its[0] < its[1]
    # a tolerance per instance is required, each finite and >= 0
    with pytest.raises(P.MipdhgError):
        P.solve_batched(P.DeviceBatch.from_lps([lp, lp]), [1e-4, float("nan")], "fp64")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_launch_split_narrow_class_bitwise_wide_class_to_tolerance(prec):
    # sizes 20..2,000 rows: the 4, 8, 16 KB budgets put instances in both launches,
    # 48 KB (above the largest instance's vectors) puts them all in the narrow one
    lps = [lpgen.cfg4_instance(700 + i, m) for i, m in enumerate(_sizes(48, 20, 2000, seed=5))]
    batch = P.DeviceBatch.from_lps(lps)
    ts = 8 if prec == "fp64" else 4
    eps = 1e-4
    ref = P.solve_batched(batch, eps, prec)
    for split in (4096, 8192, 16384, 49152):
        got = P.solve_batched(batch, eps, prec, batch_split=split)
        assert got.status == ref.status == 0
        for i, lp in enumerate(lps):
            g, r = got.split(batch, i), ref.split(batch, i)
            if (lp.m + lp.n) * ts + 16 <= split:  # narrow: the single launch's arithmetic
                assert torch.equal(g["x"], r["x"]) and torch.equal(g["y"], r["y"]), (split, i)
                assert g["info"]["iters"] == r["info"]["iters"], (split, i)
            else:  # wide: other sum partitions, the same tests met
                assert g["info"]["status"] == 0
                assert _tests_hold(lp, _np(g["x"]), _np(g["y"]), eps), (split, i)
                err, bound = objective_bound(lp, _np(g["x"]), _np(g["y"]))
                assert err <= bound * (1 + 1e-9) + 1e-12, (split, i)


def test_batched_autotuner_choice_is_parity_equal():
    lps = [lpgen.cfg4_instance(800 + i, m) for i, m in enumerate(_sizes(64, 20, 2000, seed=6))]
    batch = P.DeviceBatch.from_lps(lps)
    eps = 1e-4
    best = P.autotune_batched(batch, eps, "fp32")
    assert best["batch_split"] in (0, 2048, 4096, 8192, 16384, 32768) and best["ms"] > 0
    a = P.solve_batched(batch, eps, "fp32", batch_split=best["batch_split"])
    assert a.status == 0
    for i, lp in enumerate(lps):
        x, y = _np(a.split(batch, i)["x"]), _np(a.split(batch, i)["y"])
        assert _tests_hold(lp, x, y, eps), i
    # and the chosen run against the oracle on a few instances
    for i in (0, 31, 63):
        lp = lps[i]
        ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, eps)
        assert abs(a.infos[i]["pobj"] - ref.meas.pobj) <= 1e-3 * (1 + abs(ref.meas.pobj))


@pytest.mark.parametrize("prec,split", [("fp32", 0), ("fp64", 0), ("fp32", 4096)])
def test_resumable_blocks_give_the_one_shot_result(prec, split):
    # blocks of 128 iterations (two evaluations), resumed until every instance
    # has finished: bitwise the uninterrupted solve, instance by instance
    lps = [lpgen.cfg4_instance(900 + i, m) for i, m in enumerate(_sizes(32, 20, 1500, seed=7))]
    batch = P.DeviceBatch.from_lps(lps)
    eps = 1e-4
    ref = P.solve_batched(batch, eps, prec, batch_split=split)
    assert ref.status == 0
    sol = P.solve_batched(batch, eps, prec, batch_split=split, batch_block_iters=128)
    assert sol.status == P.IN_PROGRESS
    first = [inf["status"] for inf in sol.infos]
    assert first.count(P.IN_PROGRESS) > 0 and all(s in (0, P.IN_PROGRESS) for s in first)
    for inf in sol.infos:  # a suspended instance stopped at the first evaluation past the block
        assert inf["status"] == 0 or inf["iters"] == 128
    calls = 1
    while sol.status == P.IN_PROGRESS:
        sol = P.solve_batched(batch, eps, prec, resume=sol, batch_split=split, batch_block_iters=128)
        calls += 1
        assert calls <= 200
    assert calls == 1 + (max(inf["iters"] for inf in ref.infos) - 1) // 128
    assert sol.status == 0
    for key in ("x", "y", "z", "r_p", "r_d"):
        assert torch.equal(getattr(sol, key), getattr(ref, key)), key
    for a, b in zip(sol.infos, ref.infos):
        assert (a["status"], a["iters"], a["restarts"]) == (b["status"], b["iters"], b["restarts"])
        assert a["omega"] == b["omega"] and a["pobj"] == b["pobj"]


def test_resume_refuses_a_workspace_without_this_batchs_state():
    lps = [lpgen.cfg4_instance(950 + i, m) for i, m in enumerate([30, 80, 200])]
    batch = P.DeviceBatch.from_lps(lps)
    ref = P.solve_batched(batch, 1e-4, "fp64")
    first = P.solve_batched(batch, 1e-4, "fp64", batch_block_iters=64)
    assert first.status == P.IN_PROGRESS
    # a zeroed workspace holds no state
    blank = P.BatchSolution(0, first.x.clone(), first.y.clone(), first.z.clone(), first.r_p.clone(),
                            first.r_d.clone(), [], torch.zeros_like(first.workspace))
    with pytest.raises(P.MipdhgError) as e:
        P.solve_batched(batch, 1e-4, "fp64", resume=blank, batch_block_iters=64)
    assert e.value.code == -1
    # the state of the batch under other options
    with pytest.raises(P.MipdhgError) as e:
        P.solve_batched(batch, 1e-4, "fp64", resume=first, batch_block_iters=64, ruiz_iters=5)
    assert e.value.code == -1
    # the refused calls left the state as it was: resuming it gives the one-shot result
    sol, calls = first, 1
    while sol.status == P.IN_PROGRESS:
        sol = P.solve_batched(batch, 1e-4, "fp64", resume=sol, batch_block_iters=64)
        calls += 1
        assert calls <= 500
    assert torch.equal(sol.x, ref.x) and torch.equal(sol.y, ref.y)
    assert [i["iters"] for i in sol.infos] == [i["iters"] for i in ref.infos]


def test_resume_takes_a_new_tolerance():
    # eps_rel may change between calls: a first block at 1e-4 in which no
    # instance finishes, then the rest at 1e-6, is the one-shot 1e-6 solve
    lps = [lpgen.cfg4_instance(980 + i, m) for i, m in enumerate(_sizes(12, 100, 600, seed=8))]
    batch = P.DeviceBatch.from_lps(lps)
    ref = P.solve_batched(batch, 1e-6, "fp64")
    assert ref.status == 0
    sol = P.solve_batched(batch, 1e-4, "fp64", batch_block_iters=64)
    assert all(inf["status"] == P.IN_PROGRESS and inf["iters"] == 64 for inf in sol.infos)
    calls = 1
    while sol.status == P.IN_PROGRESS:
        sol = P.solve_batched(batch, 1e-6, "fp64", resume=sol, batch_block_iters=256)
        calls += 1
        assert calls <= 500
    assert torch.equal(sol.x, ref.x) and torch.equal(sol.y, ref.y) and torch.equal(sol.z, ref.z)
    assert [i["iters"] for i in sol.infos] == [i["iters"] for i in ref.infos]


@pytest.mark.parametrize("prec", ["bf16", "fp32acc32"])
def test_batched_reduced_precision_modes_reach_tolerance(prec):
    # BF16 matrix values (the iteration is anchor-relative, so their
    # rounding only scales the epoch's movement), and FP32 sums: every
    # instance meets the Section 2 tests when re-measured in float64 on the
    # host, with the planted-KKT objective bound
    lps = [lpgen.cfg4_instance(1100 + i, m) for i, m in enumerate(_sizes(24, 20, 1000, seed=9))]
    batch = P.DeviceBatch.from_lps(lps)
    eps = 1e-4
    sol = P.solve_batched(batch, eps, prec, max_iter=200_000)
    assert sol.status == 0
    for i, lp in enumerate(lps):
        got = sol.split(batch, i)
        x, y = _np(got["x"]), _np(got["y"])
        assert _tests_hold(lp, x, y, eps), (prec, i)
        err, bound = objective_bound(lp, x, y)
        assert err <= bound * (1 + 1e-9) + 1e-12, (prec, i, err, bound)


def test_batched_refuses_fp32a():
    batch = P.DeviceBatch.from_lps([lpgen.cfg4_instance(1200, 40)])
    with pytest.raises(P.MipdhgError) as e:
        P.solve_batched(batch, 1e-4, "fp32a")
    assert e.value.code == -6


def test_batched_extreme_instance_sizes():
    # a one-row simplex LP (optimum min_j c_j), a dense 4 x 10 instance and one
    # of 10,000 x 25,000 (140 KB of vectors in LDS, near the 150 KB limit) in
    # one FP32 launch; the same batch in FP64 needs twice that LDS: refused
    simplex = lpgen.simplex_lp(np.array([0.7, -0.3, 1.2, 0.4]))
    lps = [simplex, lpgen.cfg4_instance(1300, 4), lpgen.cfg4_instance(1301, 10000)]
    batch = P.DeviceBatch.from_lps(lps)
    eps = 1e-4
    sol = P.solve_batched(batch, eps, "fp32", max_iter=200_000)
    assert sol.status == 0
    for i, lp in enumerate(lps):
        got = sol.split(batch, i)
        x, y = _np(got["x"]), _np(got["y"])
        assert _tests_hold(lp, x, y, eps), i
        err, bound = objective_bound(lp, x, y)
        assert err <= bound * (1 + 1e-9) + 1e-12, (i, err, bound)
    assert abs(sol.infos[0]["pobj"] - (-0.3)) <= 1e-3
    with pytest.raises(P.MipdhgError) as e:
        P.solve_batched(batch, eps, "fp64")
    assert e.value.code == -6
