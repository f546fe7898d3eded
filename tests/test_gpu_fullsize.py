"""Parity at the full sizes, in the launch configuration bench.py times (the tile shapes
mipdhg_autotune picks for each LP and precision).

The oracle cannot iterate the full LPs in a test's time, but it can recompute
any single entry of one PDHG step from the previous iterate: the GPU's own
iterate after iteration 1 (exported by the trace) is fed to the oracle's step
(its own float64 scaling of the caller's matrix, the step sizes the GPU
reports), and a random sample of the entries of iteration 2 — x_hat and the
Halpern state on sampled columns, y_hat on sampled rows — is compared.
FP64 to 1e-10, float32 iterates (float32 matrix values) to 1e-5, BF16
matrix values (the oracle's step on its scaled matrix rounded to BF16) to
1e-5.  The
general-form LP of the benchmark is checked the same way with its bound and
sign projections.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import lpgen
from oracle.pdhg import scale

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_03150_amd")
torch = pytest.importorskip("torch")

_LPS = {}
_SHAPES = {}
_KEYS = ("spmv_kind", "tile_nnz", "tile_rows", "short_row", "tile_nnz_at", "tile_rows_at", "short_row_at")


def _lp(name):
    if name not in _LPS:
        _LPS[name] = {"power_law": lpgen.cfg2, "block_angular": lpgen.cfg3, "general": lpgen.general_cfg2}[name](0)
    return _LPS[name]


def _tuned(name, prec):
    """The shape mipdhg_autotune picks for this LP and precision: the launch
    configuration bench.py times (its CU-balanced tile sizes included)."""
    if (name, prec) not in _SHAPES:
        best = P.autotune(P.DeviceLP.from_lp(_lp(name)), prec, iters=64)
        _SHAPES[(name, prec)] = {k: best[k] for k in _KEYS}
    return _SHAPES[(name, prec)]


def _bf16(v):
    """Round to bfloat16 (nearest even) through float32, as the library does."""
    u = np.asarray(v, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b)) / max(1e-300, float(np.linalg.norm(b)))


def _one_step_check(lp, prec, shape, tol, samples=3000, seed=0):
    dlp = P.DeviceLP.from_lp(lp)
    sol = P.solve(dlp, 1e-12, prec, trace_iters=2, max_iter=2, **shape)
    tr = {k: _np(v) for k, v in sol.trace.items()}
    d_row, d_col, At = scale(lp.A)
    assert _rel(_np(sol.d_row), d_row) <= 1e-12 and _rel(_np(sol.d_col), d_col) <= 1e-12
    if prec == "bf16":  # the matrix the iteration applies: scaled values rounded to BF16
        At = At.copy()
        At.data = _bf16(At.data)
    bt, ct = d_row * lp.b, d_col * lp.c
    info = sol.info
    tau, sig = info["eta"] / info["omega0"], info["eta"] * info["omega0"]
    x1, y1 = tr["x"][0], tr["y"][0]
    AtT = sp.csr_matrix(At.T)
    rng = np.random.default_rng(seed)
    # x_hat and the state on sampled columns (k = 1: Halpern weight 2/3, anchor 0)
    J = rng.choice(lp.n, size=min(samples, lp.n), replace=False)
    lo_t = np.zeros(lp.n) if lp.lo is None else lp.lo / d_col
    hi_t = np.full(lp.n, np.inf) if lp.hi is None else lp.hi / d_col

    def proj_x(v, idx):
        return np.minimum(np.maximum(v, lo_t[idx]), hi_t[idx])

    def proj_y(v, idx):
        if lp.sense is None:
            return v
        s_ = lp.sense[idx]
        return np.where(s_ == 1, np.maximum(v, 0.0), np.where(s_ == 2, np.minimum(v, 0.0), v))

    xh = proj_x(x1[J] - tau * (ct[J] - AtT[J] @ y1), J)
    assert _rel(tr["xhat"][1][J], xh) <= tol
    w = 2.0 / 3.0
    assert _rel(tr["x"][1][J], w * (2.0 * xh - x1[J])) <= tol
    # y_hat on sampled rows: x_bar on the columns those rows touch
    I = rng.choice(lp.m, size=min(samples, lp.m), replace=False)
    rows = At[I]
    cols = np.unique(rows.indices)
    xh_c = proj_x(x1[cols] - tau * (ct[cols] - AtT[cols] @ y1), cols)
    xbar = np.zeros(lp.n)
    xbar[cols] = 2.0 * xh_c - x1[cols]
    yh = proj_y(y1[I] + sig * (bt[I] - rows @ xbar), I)
    assert _rel(tr["yhat"][1][I], yh) <= tol


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5), ("bf16", 1e-5)])
def test_one_step_parity_full_power_law(prec, tol):
    _one_step_check(_lp("power_law"), prec, _tuned("power_law", prec), tol)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5), ("bf16", 1e-5)])
def test_one_step_parity_full_block_angular(prec, tol):
    _one_step_check(_lp("block_angular"), prec, _tuned("block_angular", prec), tol)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_one_step_parity_full_general_power_law(prec, tol):
    # the general-form leg of the benchmark: bounds and row senses on the power-law shape
    _one_step_check(_lp("general"), prec, _tuned("general", prec), tol)


@pytest.mark.parametrize("name", ["power_law", "block_angular"])
def test_full_solve_remeasured_on_the_host(name):
    """A full-size FP32 solve to 1e-4 at the tuned shape, its point re-measured
    in float64 on the host (SciPy, original model): the three tests of
    Section 2 hold, and the GPU's own evaluation (k_eval, and k_decide's
    fixed-order reduction over thousands of partial rows) reports the same
    measures."""
    lp = _lp(name)
    sol = P.solve(P.DeviceLP.from_lp(lp), 1e-4, "fp32", **_tuned(name, "fp32"))
    assert sol.status == 0
    x, y = _np(sol.x), _np(sol.y)
    g = lp.c - lp.AT @ y
    z = np.maximum(g, 0.0)
    rp, rd = lp.b - lp.A @ x, g - z
    p, d = float(lp.c @ x), float(lp.b @ y)
    rel = (np.linalg.norm(rp) / (1 + np.linalg.norm(lp.b)), np.linalg.norm(rd) / (1 + np.linalg.norm(lp.c)),
           abs(p - d) / (1 + abs(p) + abs(d)))
    assert max(rel) <= 1e-4
    info = sol.info
    for got, ref in zip((info["rel_rp"], info["rel_rd"], info["rel_gap"]), rel):
        assert abs(got - ref) <= 1e-8 * ref + 1e-15, (got, ref)
    assert abs(info["pobj"] - p) <= 1e-12 * (1 + abs(p)) and abs(info["dobj"] - d) <= 1e-12 * (1 + abs(d))
    assert np.allclose(_np(sol.z), z, rtol=0, atol=1e-12 * (1 + np.abs(z).max()))
