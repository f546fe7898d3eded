"""Parity at the full sizes, in the launch configuration bench.py times.

The oracle cannot iterate the full LPs in a test's time, but it can recompute
any single entry of one PDHG step from the previous iterate: the GPU's own
iterate after iteration 1 (exported by the trace) is fed to the oracle's step
(its own float64 scaling of the caller's matrix, the step sizes the GPU
reports), and a random sample of the entries of iteration 2 — x_hat and the
Halpern state on sampled columns, y_hat on sampled rows — is compared.
FP64 to 1e-10, float32 iterates (float32 matrix values) to 1e-5.  The
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

# the shapes the autotuner picks for these LPs (A's tiles, then A^T's)
SHAPES = {"power_law": dict(spmv_kind=0, tile_nnz=2048, tile_rows=512, short_row=-1, tile_nnz_at=2048,
                            tile_rows_at=256, short_row_at=32),
          "block_angular": dict(spmv_kind=0, tile_nnz=8192, tile_rows=512, short_row=32, tile_nnz_at=4096,
                                tile_rows_at=512, short_row_at=32)}


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


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_one_step_parity_full_power_law(prec, tol):
    _one_step_check(lpgen.cfg2(0), prec, SHAPES["power_law"], tol)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_one_step_parity_full_block_angular(prec, tol):
    _one_step_check(lpgen.cfg3(0), prec, SHAPES["block_angular"], tol)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_one_step_parity_full_general_power_law(prec, tol):
    # the general-form leg of the benchmark: bounds and row senses on the power-law shape
    _one_step_check(lpgen.general_cfg2(0), prec, SHAPES["power_law"], tol)
