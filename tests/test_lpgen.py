"""The synthetic workloads have the stated shapes and a planted KKT point."""
import numpy as np
import scipy.sparse as sp

import lpgen


def _kkt(lp):
    assert np.abs(lp.A @ lp.x_star - lp.b).max() <= 1e-12 * max(1, np.abs(lp.b).max())
    assert np.abs(lp.AT @ lp.y_star + lp.z_star - lp.c).max() <= 1e-12 * max(1, np.abs(lp.c).max())
    assert np.all(lp.x_star >= 0) and np.all(lp.z_star >= 0)
    assert float(lp.x_star @ lp.z_star) == 0.0
    assert int((lp.x_star > 0).sum()) == lp.n // 2
    assert (lp.AT != lp.A.T).nnz == 0


def test_cfg1_shape_and_kkt():
    lp = lpgen.cfg1(0)
    assert (lp.m, lp.n, lp.nnz) == (200, 500, 2500)
    assert np.all(np.diff(lp.AT.indptr) == 5)
    _kkt(lp)
    again = lpgen.cfg1(0)
    assert np.array_equal(lp.A.data, again.A.data) and np.array_equal(lp.b, again.b)


def test_cfg2_sub_powerlaw():
    lp = lpgen.cfg2_sub(0, scale=20)  # m=5000, n=20000
    k = np.diff(lp.AT.indptr)
    assert k.min() >= 2 and k.max() <= 2000
    assert 6.5 < k.mean() < 9.5
    _kkt(lp)


def test_powerlaw_counts_mean():
    k = lpgen.powerlaw_counts(400_000, lpgen.rng_for(123))
    assert abs(k.mean() - 8.0) < 0.15 and k.min() == 2 and int(np.median(k)) == 3


def test_cfg3_small_structure():
    lp = lpgen.cfg3(nblocks=4, bm=300, bn=1200, nlink=20, link_nnz=12)
    assert lp.m == 4 * 300 + 20 and lp.n == 4 * 1200
    rl = np.diff(lp.A.indptr)
    assert np.all(rl[-20:] == 12)
    # block rows only touch their own block's columns
    A = lp.A.tocoo()
    blk = A.row < 1200
    assert np.all(A.row[blk] // 300 == A.col[blk] // 1200)
    _kkt(lp)


def test_cfg4_sizes_and_instance():
    s = lpgen.cfg4_sizes(4096)
    assert s.min() >= 20 and s.max() <= 2000
    assert 150 < np.median(s) < 260
    lp = lpgen.cfg4_instance(7, 50)
    assert (lp.m, lp.n) == (50, 125) and np.all(np.diff(lp.AT.indptr) == 4)
    _kkt(lp)


def test_stack_batch():
    lps = [lpgen.cfg4_instance(i, m) for i, m in enumerate([20, 33, 41])]
    bt = lpgen.stack_batch(lps)
    assert bt.A.shape == (94, sum(lp.n for lp in lps)) and list(bt.row_off) == [0, 20, 53, 94]
    x = np.concatenate([lp.x_star for lp in lps])
    assert np.abs(bt.A @ x - bt.b).max() < 1e-12


def test_off_block_pair_breaks_only_the_block_structure():
    ob = lpgen.off_block_pair()
    assert abs(sp.csr_matrix(ob.A.T) - ob.AT).max() == 0.0
    assert np.array_equal(ob.A.indptr[ob.row_off], ob.nnz_off)
    assert np.array_equal(ob.AT.indptr[ob.col_off], ob.nnz_off)
    A = ob.A.tocoo()
    inst_r = np.searchsorted(ob.row_off, A.row, side="right") - 1
    inst_c = np.searchsorted(ob.col_off, A.col, side="right") - 1
    assert int(np.sum(inst_r != inst_c)) == 2
