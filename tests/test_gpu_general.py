"""GPU parity of the general form (bounds l <= x <= u, rows of sense =, >=
or <=) against the float64 oracle.

FP64 per-iterate parity over 100 iterations (1e-10 relative) on several
shapes and both tile kernels; full solves with the oracle's status,
iteration and restart counts; the returned z, r_p, r_d and the dual
objective re-measured on the host from their definitions; FP32 solves to
1e-4 re-measured in float64; the general kernels given the standard bounds
reproduce the standard-form kernels bit for bit; invalid bounds and senses
are refused.
"""
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


def _gen(lp):
    return dict(lo=lp.lo, hi=lp.hi, sense=lp.sense)


def _trace_parity(lp, T=100, eval_every=64, **kw):
    dlp = P.DeviceLP.from_lp(lp)
    sol = P.solve(dlp, 1e-12, "fp64", trace_iters=T, max_iter=T, eval_every=eval_every, **kw)
    ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-12, opts=OracleOptions(max_iter=T, eval_every=eval_every),
                       trace_iters=T, **_gen(lp))
    assert sol.status == ref.status
    assert abs(sol.info["sigma_hat"] - ref.sigma_hat) <= 1e-12 * ref.sigma_hat
    tr = {k: _np(v) for k, v in sol.trace.items()}
    for t in range(1, min(T, ref.iters) + 1):
        xs, ys, xh, yh = ref.trace[t]
        for key, r in (("x", xs), ("y", ys), ("xhat", xh), ("yhat", yh)):
            e = _rel(tr[key][t - 1], r)
            assert e <= 1e-10, (t, key, e)
    return sol, ref


def _partial(lp, keep_bounds, keep_sense):
    """The same data with only the bounds or only the senses (the other part
    at its standard default)."""
    return lpgen.LP(lp.A, lp.AT, lp.b, lp.c, lp.x_star, lp.y_star, lp.z_star, name=lp.name + "_part",
                    lo=lp.lo if keep_bounds else None, hi=lp.hi if keep_bounds else None,
                    sense=lp.sense if keep_sense else None)


@pytest.mark.parametrize("make", [lambda: lpgen.general_cfg1(0), lambda: lpgen.general_cfg2_sub(0, 100),
                                  lambda: lpgen.general_tiny(12, 30, 3, 1)])
@pytest.mark.parametrize("spmv_kind", [0, 2])
def test_trace_parity_general(make, spmv_kind):
    _trace_parity(make(), spmv_kind=spmv_kind)


@pytest.mark.parametrize("bounds,sense", [(True, False), (False, True)])
def test_trace_parity_bounds_only_and_senses_only(bounds, sense):
    lp = _partial(lpgen.general_cfg1(1), bounds, sense)
    dlp = P.DeviceLP.from_lp(lp)
    assert (dlp.lo is not None) == bounds and (dlp.sense is not None) == sense
    T = 100
    sol = P.solve(dlp, 1e-12, "fp64", trace_iters=T, max_iter=T)
    kw = dict(lo=lp.lo, hi=lp.hi) if bounds else dict(sense=lp.sense)
    ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-12, opts=OracleOptions(max_iter=T), trace_iters=T, **kw)
    for t in range(1, T + 1):
        xs, ys, xh, yh = ref.trace[t]
        assert _rel(_np(sol.trace["x"][t - 1]), xs) <= 1e-10
        assert _rel(_np(sol.trace["y"][t - 1]), ys) <= 1e-10


def test_trace_parity_general_small_tiles_and_eval_every_one():
    _trace_parity(lpgen.general_cfg2_sub(1, 200), T=70, tile_nnz=256, tile_rows=64, short_row=4)
    _trace_parity(lpgen.general_tiny(8, 20, 3, 4), T=40, eval_every=1)


def _remeasure(lp, x, y):
    """The general-form quantities from their definitions, on the host."""
    Ax, g = lp.A @ x, lp.c - lp.AT @ y
    r = lp.b - Ax
    rp = np.where(lp.sense == 1, np.maximum(r, 0), np.where(lp.sense == 2, np.minimum(r, 0), r))
    lf, uf = np.isfinite(lp.lo), np.isfinite(lp.hi)
    z = np.where(lf & uf, g, np.where(lf, np.maximum(g, 0), np.where(uf, np.minimum(g, 0), 0.0)))
    rd = g - z
    lo0, hi0 = np.where(lf, lp.lo, 0.0), np.where(uf, lp.hi, 0.0)
    dobj = lp.b @ y + lo0 @ np.maximum(z, 0) - hi0 @ np.maximum(-z, 0)
    return z, rp, rd, dobj


@pytest.mark.parametrize("eps", [1e-4, 1e-8])
def test_general_solve_fp64_matches_oracle(eps):
    lp = lpgen.general_cfg1(0)
    sol = P.solve(P.DeviceLP.from_lp(lp), eps, "fp64")
    ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, eps, **_gen(lp))
    assert sol.status == ref.status == 0
    assert sol.info["iters"] == ref.iters and sol.info["restarts"] == ref.restarts
    x, y = _np(sol.x), _np(sol.y)
    assert _rel(x, ref.meas.x) <= 1e-8 and _rel(y, ref.meas.y) <= 1e-8
    tol = 1e-15 * (1 + np.abs(x))
    assert np.all(x >= lp.lo - tol) and np.all(x <= lp.hi + tol)
    assert np.all(y[lp.sense == 1] >= 0) and np.all(y[lp.sense == 2] <= 0)
    z, rp, rd, dobj = _remeasure(lp, x, y)
    assert np.allclose(_np(sol.z), z, rtol=0, atol=1e-12)
    assert np.allclose(_np(sol.r_p), rp, rtol=0, atol=1e-12)
    assert np.allclose(_np(sol.r_d), rd, rtol=0, atol=1e-12)
    assert abs(sol.info["dobj"] - dobj) <= 1e-10 * (1 + abs(dobj))
    p = lp.c @ x
    nb, nc = np.linalg.norm(lp.b), np.linalg.norm(lp.c)
    assert np.linalg.norm(rp) <= eps * (1 + nb) and np.linalg.norm(rd) <= eps * (1 + nc)
    assert abs(p - dobj) <= eps * (1 + abs(p) + abs(dobj))
    assert abs(p - lp.p_star) <= 10 * eps * (1 + abs(lp.p_star))


def test_general_fp32_reaches_tolerance_remeasured():
    lp = lpgen.general_cfg2_sub(0, 100)
    eps = 1e-4
    sol = P.solve(P.DeviceLP.from_lp(lp), eps, "fp32")
    assert sol.status == 0
    x, y = _np(sol.x), _np(sol.y)
    z, rp, rd, dobj = _remeasure(lp, x, y)
    p = lp.c @ x
    assert np.linalg.norm(rp) <= eps * (1 + np.linalg.norm(lp.b))
    assert np.linalg.norm(rd) <= eps * (1 + np.linalg.norm(lp.c))
    assert abs(p - dobj) <= eps * (1 + abs(p) + abs(dobj))
    assert abs(p - lp.p_star) <= 100 * eps * (1 + abs(lp.p_star))


@pytest.mark.parametrize("spmv_kind", [0, 2])
def test_general_kernels_with_standard_bounds_are_bitwise_standard(spmv_kind):
    lp = lpgen.cfg1(0)
    a = P.solve(P.DeviceLP.from_lp(lp), 1e-8, "fp64", spmv_kind=spmv_kind)
    g = P.DeviceLP(lp.A, lp.AT, lp.b, lp.c, lo=np.zeros(lp.n), hi=np.full(lp.n, np.inf),
                   sense=np.zeros(lp.m, dtype=np.int8))
    b = P.solve(g, 1e-8, "fp64", spmv_kind=spmv_kind)
    assert a.info["iters"] == b.info["iters"] and a.info["restarts"] == b.info["restarts"]
    for k in ("x", "y", "z", "r_p", "r_d"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    assert a.info["dobj"] == b.info["dobj"] and a.info["xz"] == b.info["xz"]


def test_general_input_errors():
    lp = lpgen.general_cfg1(0)

    def solve_with(**kw):
        d = dict(lo=lp.lo, hi=lp.hi, sense=lp.sense)
        d.update(kw)
        return P.solve(P.DeviceLP(lp.A, lp.AT, lp.b, lp.c, **d), 1e-4, "fp64")

    bad_lo = lp.lo.copy()
    bad_lo[3] = lp.hi[3] + 1.0 if np.isfinite(lp.hi[3]) else np.inf
    for kw in (dict(lo=bad_lo), dict(lo=np.where(np.arange(lp.n) == 5, np.nan, lp.lo)),
               dict(hi=np.full(lp.n, -np.inf)), dict(sense=np.full(lp.m, 3, dtype=np.int8))):
        with pytest.raises(P.MipdhgError) as e:
            solve_with(**kw)
        assert e.value.code == -1
    with pytest.raises(P.MipdhgError) as e:
        P.solve(P.DeviceLP.from_lp(lp), 1e-4, "fp64", spmv_kind=1)
    assert e.value.code == -6
    batch = P.DeviceBatch.from_lps([lpgen.tiny(6, 15, 3, 0)])
    batch.lp.sense = torch.zeros(6, dtype=torch.int8, device=batch.lp.device)
    with pytest.raises(P.MipdhgError) as e:
        P.solve_batched(batch, 1e-4, "fp32")
    assert e.value.code == -6


def test_autotune_on_a_general_lp_picks_a_tile_shape():
    lp = lpgen.general_cfg2_sub(0, 100)
    dlp = P.DeviceLP.from_lp(lp)
    best = P.autotune(dlp, "fp32", iters=32)
    # lane groups (kind 1) do not run the general form; tiles, persistent tiles, panels do
    assert best["spmv_kind"] in (0, 2, 3) and best["ms_per_iter"] > 0
    shape = {k: v for k, v in best.items() if k not in ("ms_per_iter", "cache_hit")}
    a = P.solve(dlp, 1e-4, "fp32", **shape)
    b = P.solve(dlp, 1e-4, "fp32")
    # float32 row sums round differently with other tiles: the stopping
    # evaluation may move by a block
    assert a.status == b.status == 0 and abs(a.info["iters"] - b.info["iters"]) <= 128
    assert abs(a.info["pobj"] - b.info["pobj"]) <= 1e-3 * (1 + abs(b.info["pobj"]))
