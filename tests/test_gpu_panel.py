"""The dual step on A's panel layout (spmv_kind 3) against the oracle.

The layout groups rows of narrow column span (the blocks of a
block-structured matrix) and rows of wide span (linking rows), stages each
panel of the gathered vector in LDS and adds each row's panel sums in panel
order.  Small panel widths put the small test LPs through every part of it:
several panels per group, wide groups, chunks cut at row ends, rows without
nonzeros in a panel, empty rows.  FP64 per-iterate parity is 1e-10 as for the
other kernels; the float32 path reaches its tolerance re-measured in float64.
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


def _small_block_angular(seed=0):
    # 4 blocks 300 x 1200 (6 per column) + 20 linking rows of 60 over all columns
    return lpgen.cfg3(seed, nblocks=4, bm=300, bn=1200, nlink=20, link_nnz=60)


def _trace(lp, T=100, eval_every=64, spmv_kind=3, **kw):
    sol = P.solve(P.DeviceLP.from_lp(lp), 1e-12, "fp64", trace_iters=T, max_iter=T, eval_every=eval_every,
                  spmv_kind=spmv_kind, **kw)
    ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-12, opts=OracleOptions(max_iter=T, eval_every=eval_every),
                       trace_iters=T, lo=lp.lo, hi=lp.hi, sense=lp.sense)
    assert sol.status == ref.status
    tr = {k: _np(v) for k, v in sol.trace.items()}
    for t in range(1, min(T, ref.iters) + 1):
        xs, ys, xh, yh = ref.trace[t]
        for key, r in (("x", xs), ("y", ys), ("xhat", xh), ("yhat", yh)):
            e = _rel(tr[key][t - 1], r)
            assert e <= 1e-10, (t, key, e)


@pytest.mark.parametrize("width", [0, 512, 256])
def test_trace_parity_block_angular(width):
    # 0: one panel per block; 512: 3 panels per block, the linking rows a wide
    # group of 10 panels; 256: every row wide, 19 panels
    _trace(_small_block_angular(), panel_width=width)


def test_layout_larger_than_its_capacity_is_unsupported():
    # 64-entry panels: every row wide over 75 panels, 91,500 row parts, more
    # than the workspace reserves for this LP (5 m + nnz + 1024)
    lp = _small_block_angular()
    with pytest.raises(P.MipdhgError) as e:
        P.solve(P.DeviceLP.from_lp(lp), 1e-4, "fp64", spmv_kind=3, panel_width=64)
    assert e.value.code == -6 and "capacity" in str(e.value)


def test_trace_parity_rows_over_more_panels_than_a_wave_has_lanes():
    # 64-entry panels on 6,000 columns: the block rows span about 47 panels,
    # the linking rows 94, so a wave's lanes take two panels of those rows each
    lp = lpgen.cfg3(0, nblocks=2, bm=20, bn=3000, nlink=5, link_nnz=100)
    _trace(lp, panel_width=64)


@pytest.mark.parametrize("width", [0, 64])
def test_trace_parity_random_and_general(width):
    _trace(lpgen.cfg1(0), panel_width=width)
    _trace(lpgen.general_cfg1(1), T=70, eval_every=16, panel_width=width)


def test_trace_parity_empty_rows_and_tile_shapes():
    lp = lpgen.cfg2_sub(3, scale=400)
    _trace(lp, T=70, panel_width=128, tile_nnz_at=512, tile_rows_at=64, short_row_at=-1)


def test_full_solve_matches_oracle_and_float32_converges():
    lp = _small_block_angular(1)
    dlp = P.DeviceLP.from_lp(lp)
    a = P.solve(dlp, 1e-8, "fp64", spmv_kind=3, panel_width=256)
    ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-8)
    assert a.status == ref.status == 0 and a.info["iters"] == ref.iters
    assert a.info["restarts"] == ref.restarts
    eps = 1e-6
    s = P.solve(dlp, eps, "fp32", spmv_kind=3, panel_width=256, max_iter=200_000)
    x, y = _np(s.x), _np(s.y)
    rp = lp.b - lp.A @ x
    rd = lp.c - lp.AT @ y - np.maximum(lp.c - lp.AT @ y, 0.0)
    p, d = lp.c @ x, lp.b @ y
    assert s.status == 0
    assert np.linalg.norm(rp) <= eps * (1 + np.linalg.norm(lp.b))
    assert np.linalg.norm(rd) <= eps * (1 + np.linalg.norm(lp.c))
    assert abs(p - d) <= eps * (1 + abs(p) + abs(d))
    assert abs(p - ref.meas.pobj) <= 1e-4 * abs(ref.meas.pobj)


def test_deterministic_and_graph_equals_direct():
    lp = _small_block_angular(2)
    dlp = P.DeviceLP.from_lp(lp)
    a = P.solve(dlp, 1e-6, "fp32", spmv_kind=3, panel_width=512)
    b = P.solve(dlp, 1e-6, "fp32", spmv_kind=3, panel_width=512)
    c = P.solve(dlp, 1e-6, "fp32", spmv_kind=3, panel_width=512, use_graph=0)
    assert torch.equal(a.x, b.x) and torch.equal(a.y, b.y)
    assert torch.equal(a.x, c.x) and torch.equal(a.y, c.y)


def test_row_longer_than_a_chunk_in_one_panel_is_unsupported():
    # row 0 of A holds 2,000 nonzeros inside one panel: more than a chunk
    A = np.zeros((3, 2000))
    A[0, :] = 1.0
    A[1, :5] = 1.0
    A[2, 5:9] = 1.0
    import scipy.sparse as sp
    As = sp.csr_matrix(A)
    lp = P.DeviceLP(As, sp.csr_matrix(As.T), np.array([1.0, 0.5, 0.5]), np.ones(2000), "cuda")
    with pytest.raises(P.MipdhgError) as e:
        P.solve(lp, 1e-4, "fp64", spmv_kind=3)
    assert e.value.code == -6 and "chunk" in str(e.value) or "nonzeros in one panel" in str(e.value)
    with pytest.raises(P.MipdhgError):
        P.solve(lp, 1e-4, "fp64", spmv_kind=3, panel_width=100)  # not a power of two


# --- spmv_kind 4: the primal step on A^T's row-panel layout as well

def _six_blocks():
    # 6 blocks 300 x 400 (6 per column) + 20 linking rows of 60: with 1,024-entry panels the
    # linking rows (span 2,400 > 512) are the tail, the block rows (span 400) are not, and
    # A^T's windows (300 rows a block) group three blocks at a time
    return lpgen.cfg3(0, nblocks=6, bm=300, bn=400, nlink=20, link_nnz=60)


@pytest.mark.parametrize("width", [0, 1024])
def test_row_panels_trace_parity_block_angular(width):
    _trace(_six_blocks(), panel_width=width, spmv_kind=4)


def _with_empty_columns(lp, k=5):
    # k columns of A without nonzeros (rows of A^T that get one zero element), cost 1
    from types import SimpleNamespace
    import scipy.sparse as sp
    A = sp.hstack([lp.A, sp.csr_matrix((lp.m, k))]).tocsr()
    A.sort_indices()
    return SimpleNamespace(A=A, AT=sp.csr_matrix(A.T), b=lp.b, c=np.concatenate([lp.c, np.ones(k)]), lo=None,
                           hi=None, sense=None)


def test_row_panels_trace_parity_random_general_and_empty_columns():
    _trace(lpgen.cfg1(0), spmv_kind=4)
    _trace(lpgen.general_cfg1(1), T=70, eval_every=16, spmv_kind=4)
    _trace(_with_empty_columns(lpgen.cfg1(2)), T=70, spmv_kind=4)
    _trace(lpgen.cfg2_sub(3, scale=400), T=70, spmv_kind=4, tile_nnz_at=512, tile_rows_at=64)


def test_row_panels_full_solve_and_float32():
    lp = _six_blocks()
    dlp = P.DeviceLP.from_lp(lp)
    a = P.solve(dlp, 1e-8, "fp64", spmv_kind=4, panel_width=1024)
    ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-8)
    assert a.status == ref.status == 0 and a.info["iters"] == ref.iters
    s = P.solve(dlp, 1e-6, "fp32", spmv_kind=4, panel_width=1024, max_iter=200_000)
    b = P.solve(dlp, 1e-6, "fp32", spmv_kind=4, panel_width=1024, use_graph=0)
    assert s.status == 0 and torch.equal(s.x, b.x) and torch.equal(s.y, b.y)
    assert abs(s.info["pobj"] - ref.meas.pobj) <= 1e-4 * abs(ref.meas.pobj)
    for prec in ("bf16", "fp32"):
        c = P.solve(dlp, 1e-4, prec, spmv_kind=4)
        assert c.status == 0


def test_row_panels_refuse_a_matrix_without_the_structure():
    # 64-entry panels: every row of cfg1's A (up to 500 columns) is wide, not a short tail
    with pytest.raises(P.MipdhgError) as e:
        P.solve(P.DeviceLP.from_lp(lpgen.cfg1(0)), 1e-4, "fp64", spmv_kind=4, panel_width=64)
    assert e.value.code == -6 and "row-panel" in str(e.value)
