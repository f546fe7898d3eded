"""Seeded synthetic standard-form LPs with a planted optimum.

This module only builds inputs.  It holds none of the solver's arithmetic and
is imported by the tests and the benchmark on behalf of both the CPU oracle and
the GPU library, which never import each other.

Every instance is ``min c^T x  s.t.  A x = b, x >= 0`` (paper, Section 2).  A
planted primal-dual pair ``(x*, y*, z*)`` makes the optimum known in closed
form: ``b = A x*`` and ``c = A^T y* + z*`` with ``x* >= 0``, ``z* >= 0`` and
``x*_j z*_j = 0``, so ``p* = c^T x* = b^T y*`` (complementarity, Section 2).

Draw order per instance (one PCG64 stream per seed key):
  1. column nonzero counts, 2. distinct rows per column, 3. values,
  4. a permutation whose first floor(n/2) entries form supp(x*),
  5. x*_S ~ U(0,1), 6. y* ~ N(0,1), 7. z* ~ U(0,1) off the support,
  8. b = A x*, c = A^T y* + z* in float64.

General-form instances (``general_from_matrix``) add variable bounds
``lo <= x <= hi`` (either side may be infinite) and a sense per row
(0: ``(Ax)_i = b_i``, 1: ``>=``, 2: ``<=``), with a planted optimum that
satisfies the KKT conditions of that form.  Draw order after the matrix:
  1. a kind per column (0 [0,inf), 1 box [l, l+w], 2 free, 3 (-inf, u],
     4 [l, inf)), 2. its bounds, 3. its status (at lower, at upper or
  between) and x*_j, 4. lambda*_j with the sign its status allows, 5. a
  sense per row, 6. which inequality rows are active, 7. y* (zero on
  inactive rows, signed on active ones), 8. the slack of inactive rows;
  then b = A x* -/+ slack, c = A^T y* + lambda*.  p* = c^T x* equals the dual
  value b^T y* + sum_j (l_j lambda_j^+ - u_j lambda_j^-).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np
import scipy.sparse as sp

__all__ = [
    "LP", "rng_for", "planted_from_columns", "uniform_columns", "cfg1", "cfg2",
    "cfg2_sub", "cfg3", "cfg4_sizes", "cfg4_instance", "cfg4_batch",
    "cfg5_instance", "cfg5_batch", "cfg5_fd_instance", "tiny", "simplex_lp",
    "powerlaw_counts", "Batch", "stack_batch", "general_from_matrix", "general_tiny",
    "general_cfg1", "general_cfg2", "general_cfg2_sub", "SENSE_EQ", "SENSE_GE", "SENSE_LE",
    "farkas_tiny", "unbounded_tiny", "conflicting_rows", "unbounded_column", "box_infeasible",
]

SENSE_EQ, SENSE_GE, SENSE_LE = 0, 1, 2

POWER_ALPHA = 2.1423  # p(k) ~ k^-alpha on [2, 2000] has mean 8.0


@dataclass
class LP:
    """One standard-form LP in CSR (A) plus a CSR copy of A^T, all float64."""
    A: sp.csr_matrix
    AT: sp.csr_matrix
    b: np.ndarray
    c: np.ndarray
    x_star: np.ndarray
    y_star: np.ndarray
    z_star: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)
    lo: np.ndarray | None = None     # general form: lower bounds of x
    hi: np.ndarray | None = None     # upper bounds of x
    sense: np.ndarray | None = None  # int8 per row: 0 =, 1 >=, 2 <=

    @property
    def general(self) -> bool:
        return self.lo is not None

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]

    @property
    def nnz(self) -> int:
        return int(self.A.nnz)

    @property
    def p_star(self) -> float:
        return float(self.c @ self.x_star)


def rng_for(*key: int) -> np.random.Generator:
    """PCG64 stream keyed by a tuple of non-negative integers."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def _distinct_rows(counts: np.ndarray, m: int, rng: np.random.Generator) -> np.ndarray:
    """For column j draw counts[j] distinct row indices uniformly from [0, m).

    Returns the row indices in column-major order (column 0's rows first), each
    column's rows sorted ascending.  Duplicates inside a column are redrawn
    until none remain; the redraw order is fixed, so the result is a function
    of the generator state only.
    """
    counts = np.asarray(counts, dtype=np.int64)
    if np.any(counts > m):
        raise ValueError("a column asks for more distinct rows than m")
    n = counts.size
    nnz = int(counts.sum())
    rows = rng.integers(0, m, size=nnz, dtype=np.int64)
    if n and np.all(counts == counts[0]):
        # equal counts: sort each column's rows as a row of an (n, k) array,
        # which gives the same order as the general (column, row) sort below
        k = int(counts[0])
        r2 = rows.reshape(n, k)
        while True:
            r2.sort(axis=1)
            dup = np.zeros_like(r2, dtype=bool)
            if k > 1:
                dup[:, 1:] = r2[:, 1:] == r2[:, :-1]
            nd = int(dup.sum())
            if nd == 0:
                return r2.reshape(-1)
            r2[dup] = rng.integers(0, m, size=nd, dtype=np.int64)
    colid = np.repeat(np.arange(n, dtype=np.int64), counts)
    while True:
        order = np.lexsort((rows, colid))
        rows = rows[order]  # colid is already non-decreasing and stays so
        dup = np.zeros(nnz, dtype=bool)
        if nnz > 1:
            dup[1:] = (rows[1:] == rows[:-1]) & (colid[1:] == colid[:-1])
        nd = int(dup.sum())
        if nd == 0:
            return rows
        rows[dup] = rng.integers(0, m, size=nd, dtype=np.int64)


def _csr_pair_from_columns(m: int, n: int, counts: np.ndarray, rows: np.ndarray,
                           vals: np.ndarray) -> tuple[sp.csr_matrix, sp.csr_matrix]:
    """Column-major triplets -> (A in CSR, A^T in CSR), int32 indices, sorted."""
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=colptr[1:])
    AT = sp.csr_matrix((vals.astype(np.float64), rows.astype(np.int32),
                        colptr.astype(np.int32)), shape=(n, m))
    AT.has_sorted_indices = True
    A = AT.T.tocsr()
    A.sort_indices()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    return A, AT


def planted_from_columns(m: int, counts: np.ndarray, rows: np.ndarray,
                         vals: np.ndarray, rng: np.random.Generator,
                         name: str = "", meta: dict | None = None) -> LP:
    """Steps 4-8 of the draw order on a given sparsity pattern and values."""
    n = counts.size
    A, AT = _csr_pair_from_columns(m, n, counts, rows, vals)
    perm = rng.permutation(n)
    supp = perm[: n // 2]
    x_star = np.zeros(n)
    x_star[supp] = rng.uniform(0.0, 1.0, size=supp.size)
    y_star = rng.standard_normal(m)
    z_star = np.zeros(n)
    off = perm[n // 2:]
    z_star[off] = rng.uniform(0.0, 1.0, size=off.size)
    b = A @ x_star
    c = AT @ y_star + z_star
    return LP(A, AT, b, c, x_star, y_star, z_star, name=name, meta=dict(meta or {}))


def uniform_columns(m: int, n: int, per_col: int, rng: np.random.Generator,
                    name: str = "", meta: dict | None = None) -> LP:
    """per_col distinct uniform rows in every column, values N(0,1)."""
    counts = np.full(n, per_col, dtype=np.int64)
    rows = _distinct_rows(counts, m, rng)
    vals = rng.standard_normal(rows.size)
    return planted_from_columns(m, counts, rows, vals, rng, name=name, meta=meta)


def cfg1(seed: int = 0) -> LP:
    """m=200, n=500, 5 nonzeros per column at uniform-random rows, N(0,1)."""
    return uniform_columns(200, 500, 5, rng_for(1, seed), name=f"cfg1_s{seed}",
                           meta={"cfg": 1, "seed": seed})


def powerlaw_counts(n: int, rng: np.random.Generator, kmin: int = 2, kmax: int = 2000,
                    alpha: float = POWER_ALPHA) -> np.ndarray:
    """Discrete truncated power law p(k) ~ k^-alpha on [kmin, kmax]."""
    k = np.arange(kmin, kmax + 1)
    p = k.astype(np.float64) ** (-alpha)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    u = rng.uniform(0.0, 1.0, size=n)
    idx = np.minimum(np.searchsorted(cdf, u, side="right"), k.size - 1)
    return k[idx].astype(np.int64)


def _cfg2_like(m: int, n: int, rng: np.random.Generator, kmax: int, name: str,
               meta: dict) -> LP:
    counts = powerlaw_counts(n, rng, kmax=min(kmax, m))
    rows = _distinct_rows(counts, m, rng)
    vals = rng.standard_normal(rows.size)
    row_factor = rng.uniform(0.1, 10.0, size=m)
    vals = vals * row_factor[rows]
    return planted_from_columns(m, counts, rows, vals, rng, name=name, meta=meta)


def cfg2(seed: int = 0) -> LP:
    """m=100,000, n=400,000, power-law column counts (min 2, mean 8, max 2000),
    values N(0,1) times a per-row factor U(0.1, 10)."""
    return _cfg2_like(100_000, 400_000, rng_for(2, seed), 2000, f"cfg2_s{seed}",
                      {"cfg": 2, "seed": seed})


def cfg2_sub(seed: int = 0, scale: int = 100) -> LP:
    """The cfg2 recipe at 1/scale of its size (column counts capped at m)."""
    m, n = 100_000 // scale, 400_000 // scale
    return _cfg2_like(m, n, rng_for(2, 1000 + scale, seed), 2000,
                      f"cfg2sub{scale}_s{seed}", {"cfg": 2, "seed": seed, "scale": scale})


def cfg3(seed: int = 0, nblocks: int = 64, bm: int = 30_000, bn: int = 120_000,
         per_col: int = 6, nlink: int = 2_000, link_nnz: int = 1_200) -> LP:
    """Block-angular LP: nblocks diagonal blocks bm x bn (per_col nnz per column
    inside its block), plus nlink linking rows with link_nnz distinct columns
    each drawn over all n columns.  Values N(0,1).  The defaults give
    m = 1,922,000, n = 7,680,000 and about 48.5M nonzeros."""
    rng = rng_for(3, seed, nblocks, bm)
    m = nblocks * bm + nlink
    n = nblocks * bn
    # block part: column j of block k has per_col distinct rows in [k*bm, (k+1)*bm)
    parts = [_distinct_rows(np.full(bn, per_col, dtype=np.int64), bm, rng) + k * bm
             for k in range(nblocks)]
    block_rows = np.concatenate(parts)
    del parts
    # link rows: each picks link_nnz distinct columns among all n
    lcols = _distinct_rows(np.full(nlink, link_nnz, dtype=np.int64), n, rng)
    lrow_ids = np.repeat(np.arange(nlink, dtype=np.int64), link_nnz) + nblocks * bm
    # merge into column-major order: each column's block rows (sorted, all
    # below nblocks*bm) followed by its link rows in increasing order
    lcount = np.bincount(lcols, minlength=n).astype(np.int64)
    counts = per_col + lcount
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=colptr[1:])
    all_rows = np.empty(int(colptr[-1]), dtype=np.int64)
    pos = np.repeat(colptr[:-1], per_col) + np.tile(np.arange(per_col, dtype=np.int64), n)
    all_rows[pos] = block_rows
    del pos, block_rows
    o = np.argsort(lcols, kind="stable")
    scols = lcols[o]
    lstart = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lcount, out=lstart[1:])
    within = np.arange(scols.size, dtype=np.int64) - lstart[scols]
    all_rows[colptr[scols] + per_col + within] = lrow_ids[o]
    vals = rng.standard_normal(all_rows.size)
    return planted_from_columns(m, counts, all_rows, vals, rng, name=f"cfg3_s{seed}",
                                meta={"cfg": 3, "seed": seed, "nblocks": nblocks,
                                      "bm": bm, "bn": bn, "nlink": nlink,
                                      "link_nnz": link_nnz})


def cfg4_sizes(count: int = 4096, seed: int = 0) -> np.ndarray:
    """m_i = round(exp(U(ln 20, ln 2000))) for each instance (log-uniform)."""
    rng = rng_for(4, seed, 999_999)
    return np.rint(np.exp(rng.uniform(math.log(20), math.log(2000), size=count))).astype(np.int64)


def cfg4_instance(i: int, m: int, seed: int = 0) -> LP:
    """Instance i of the batched workload: n = round(2.5 m), 4 nnz per column."""
    n = int(round(2.5 * m))
    return uniform_columns(int(m), n, 4, rng_for(4, seed, i), name=f"cfg4_{i}",
                           meta={"cfg": 4, "seed": seed, "inst": i})


def cfg4_batch(count: int = 4096, seed: int = 0) -> list[LP]:
    sizes = cfg4_sizes(count, seed)
    return [cfg4_instance(i, int(m), seed) for i, m in enumerate(sizes)]


def cfg5_instance(i: int, seed: int = 0, m: int = 500, n: int = 1500) -> tuple[LP, np.ndarray]:
    """Differentiation workload instance and its loss weights w ~ N(0,1)^n."""
    rng = rng_for(5, seed, i)
    lp = uniform_columns(m, n, 5, rng, name=f"cfg5_{seed}_{i}",
                         meta={"cfg": 5, "seed": seed, "inst": i})
    w = rng.standard_normal(n)
    return lp, w


def cfg5_batch(count: int = 256, seed: int = 0) -> tuple[list[LP], list[np.ndarray]]:
    lps, ws = [], []
    for i in range(count):
        lp, w = cfg5_instance(i, seed)
        lps.append(lp)
        ws.append(w)
    return lps, ws


def cfg5_fd_instance(i: int) -> tuple[LP, np.ndarray]:
    """The small finite-difference set: m=20, n=50, 5 nnz per column."""
    return cfg5_instance(i, seed=1, m=20, n=50)


def tiny(m: int, n: int, per_col: int, seed: int) -> LP:
    """Small planted LPs for brute-force checks."""
    return uniform_columns(m, n, min(per_col, m), rng_for(9, m, n, per_col, seed),
                           name=f"tiny_{m}x{n}_s{seed}")


def simplex_lp(c: np.ndarray) -> LP:
    """m = 1: sum(x) = 1, x >= 0.  The optimum is min_j c_j (textbook)."""
    n = c.size
    counts = np.ones(n, dtype=np.int64)
    rows = np.zeros(n, dtype=np.int64)
    vals = np.ones(n)
    A, AT = _csr_pair_from_columns(1, n, counts, rows, vals)
    j = int(np.argmin(c))
    x = np.zeros(n)
    x[j] = 1.0
    y = np.array([c[j]])
    z = c - c[j]
    return LP(A, AT, np.array([1.0]), c.astype(np.float64), x, y, z, name="simplex")


def slow_power_lp(seed: int = 0) -> LP:
    """A 3 x 201 LP on which 100 power iterations of the scaled matrix have not
    settled: [1] beside a 2 x 200 all-ones block with six entries negated.
    After scaling the lone entry is a singular value 1 whose singular vector
    holds weight 1/sqrt(201) of the uniform start, and the block's largest
    singular value is about 0.985.  Planted optimum as elsewhere."""
    B2 = np.ones((2, 200))
    for k in range(6):
        B2[k % 2, (7 * k) % 200] = -1.0
    A = sp.csr_matrix(sp.block_diag([np.ones((1, 1)), B2]))
    A.sort_indices()
    rng = rng_for(10, seed)
    m, n = A.shape
    x = np.zeros(n)
    supp = rng.permutation(n)[: n // 2]
    x[supp] = rng.uniform(0.0, 1.0, supp.size)
    y = rng.normal(size=m)
    z = np.where(x > 0, 0.0, rng.uniform(0.0, 1.0, n))
    AT = sp.csr_matrix(A.T)
    AT.sort_indices()
    return LP(A, AT, A @ x, AT @ y + z, x, y, z, name=f"slow_power_s{seed}")


def off_block_pair() -> "Batch":
    """Two stacked instances (m = 25) whose A, and its exact transpose, carry
    one entry of instance 0 in instance 1's columns and one of instance 1 in
    instance 0's: row pointers, nonzero offsets and A^T = A^T all hold, only
    the block-diagonal structure is broken (an invalid batch for validation
    tests)."""
    lps = [cfg4_instance(500 + i, 25) for i in range(2)]
    good = stack_batch(lps)
    ro, co = good.row_off, good.col_off
    A = good.A.tocoo()
    r, c, v = A.row.copy(), A.col.copy(), A.data.copy()
    k0 = int(np.flatnonzero(r < ro[1])[0])
    k1 = int(np.flatnonzero(r >= ro[1])[0])
    used0 = set(c[r == r[k0]].tolist())
    used1 = set(c[r == r[k1]].tolist())
    c[k0] = next(j for j in range(co[1], co[2]) if j not in used0)
    c[k1] = next(j for j in range(co[0], co[1]) if j not in used1)
    Ab = sp.csr_matrix((v, (r, c)), shape=A.shape)
    Ab.sort_indices()
    ATb = sp.csr_matrix(Ab.T)
    ATb.sort_indices()
    return Batch(Ab, ATb, good.b, good.c, good.row_off, good.col_off, good.nnz_off, lps)


@dataclass
class Batch:
    """Block-diagonal stacking of independent LPs (global column indices)."""
    A: sp.csr_matrix
    AT: sp.csr_matrix
    b: np.ndarray
    c: np.ndarray
    row_off: np.ndarray  # int32 [B+1]
    col_off: np.ndarray  # int32 [B+1]
    nnz_off: np.ndarray  # int64 [B+1]
    lps: list

    @property
    def B(self) -> int:
        return len(self.lps)


def stack_batch(lps: list[LP]) -> Batch:
    A = sp.block_diag([lp.A for lp in lps], format="csr")
    A.sort_indices()
    AT = sp.block_diag([lp.AT for lp in lps], format="csr")
    AT.sort_indices()
    for M in (A, AT):
        M.indices = M.indices.astype(np.int32)
        M.indptr = M.indptr.astype(np.int32)
    row_off = np.zeros(len(lps) + 1, dtype=np.int32)
    col_off = np.zeros(len(lps) + 1, dtype=np.int32)
    nnz_off = np.zeros(len(lps) + 1, dtype=np.int64)
    row_off[1:] = np.cumsum([lp.m for lp in lps])
    col_off[1:] = np.cumsum([lp.n for lp in lps])
    nnz_off[1:] = np.cumsum([lp.nnz for lp in lps])
    b = np.concatenate([lp.b for lp in lps])
    c = np.concatenate([lp.c for lp in lps])
    return Batch(A, AT, b, c, row_off, col_off, nnz_off, list(lps))


def general_from_matrix(A: sp.csr_matrix, AT: sp.csr_matrix, rng: np.random.Generator,
                        name: str = "", meta: dict | None = None,
                        kind_p=(0.3, 0.25, 0.1, 0.15, 0.2), sense_p=(0.5, 0.25, 0.25)) -> LP:
    """A general-form LP on the given matrix with a planted KKT point (draw
    order in the module docstring).  z_star holds the planted reduced costs
    lambda* (signed)."""
    m, n = A.shape
    kind = rng.choice(5, size=n, p=list(kind_p))
    lo = np.zeros(n)
    hi = np.full(n, np.inf)
    box = kind == 1
    lo[box] = rng.uniform(-1.0, 0.0, size=int(box.sum()))
    hi[box] = lo[box] + rng.uniform(0.5, 2.0, size=int(box.sum()))
    free = kind == 2
    lo[free], hi[free] = -np.inf, np.inf
    up = kind == 3
    lo[up] = -np.inf
    hi[up] = rng.uniform(-1.0, 1.0, size=int(up.sum()))
    low = kind == 4
    lo[low] = rng.uniform(-1.0, 1.0, size=int(low.sum()))
    # status: 0 at lower, 1 at upper, 2 between
    u = rng.uniform(0.0, 1.0, size=n)
    status = np.where(kind == 0, np.where(u < 0.5, 0, 2),
                      np.where(kind == 1, np.where(u < 1 / 3, 0, np.where(u < 2 / 3, 1, 2)),
                               np.where(kind == 2, 2,
                                        np.where(kind == 3, np.where(u < 0.5, 1, 2),
                                                 np.where(u < 0.5, 0, 2)))))
    t = rng.uniform(0.0, 1.0, size=n)
    g = rng.standard_normal(n)
    x = np.empty(n)
    x[status == 0] = lo[status == 0]
    x[status == 1] = hi[status == 1]
    mid = status == 2
    fin = np.isfinite(lo) & np.isfinite(hi)
    x[mid & fin] = lo[mid & fin] + t[mid & fin] * (hi[mid & fin] - lo[mid & fin])
    only_lo = mid & np.isfinite(lo) & ~np.isfinite(hi)
    x[only_lo] = lo[only_lo] + t[only_lo]
    only_hi = mid & ~np.isfinite(lo) & np.isfinite(hi)
    x[only_hi] = hi[only_hi] - t[only_hi]
    fr = mid & ~np.isfinite(lo) & ~np.isfinite(hi)
    x[fr] = g[fr]
    lam_mag = rng.uniform(0.0, 1.0, size=n)
    lam = np.where(status == 0, lam_mag, np.where(status == 1, -lam_mag, 0.0))
    sense = rng.choice(3, size=m, p=list(sense_p)).astype(np.int8)
    active = rng.uniform(0.0, 1.0, size=m) < 0.6
    ymag = rng.uniform(0.0, 1.0, size=m)
    yn = rng.standard_normal(m)
    y = np.where(sense == SENSE_EQ, yn,
                 np.where(active, np.where(sense == SENSE_GE, ymag, -ymag), 0.0))
    slack = rng.uniform(0.1, 1.0, size=m)
    b = A @ x
    ina = (sense != SENSE_EQ) & ~active
    b[ina & (sense == SENSE_GE)] -= slack[ina & (sense == SENSE_GE)]
    b[ina & (sense == SENSE_LE)] += slack[ina & (sense == SENSE_LE)]
    c = AT @ y + lam
    return LP(A, AT, b, c, x, y, lam, name=name, meta=dict(meta or {}), lo=lo, hi=hi, sense=sense)


def _matrix_uniform(m: int, n: int, per_col: int, rng: np.random.Generator):
    counts = np.full(n, per_col, dtype=np.int64)
    rows = _distinct_rows(counts, m, rng)
    vals = rng.standard_normal(rows.size)
    return _csr_pair_from_columns(m, n, counts, rows, vals)


def general_tiny(m: int, n: int, per_col: int, seed: int) -> LP:
    """Small general-form LPs for exact checks."""
    rng = rng_for(11, m, n, per_col, seed)
    A, AT = _matrix_uniform(m, n, min(per_col, m), rng)
    return general_from_matrix(A, AT, rng, name=f"gtiny_{m}x{n}_s{seed}")


def general_cfg1(seed: int = 0) -> LP:
    """The small workload's matrix (200 x 500, 5 per column) in general form."""
    rng = rng_for(12, seed)
    A, AT = _matrix_uniform(200, 500, 5, rng)
    return general_from_matrix(A, AT, rng, name=f"gcfg1_s{seed}", meta={"cfg": 1, "seed": seed})


def _cfg2_matrix(m: int, n: int, rng: np.random.Generator, kmax: int):
    counts = powerlaw_counts(n, rng, kmax=min(kmax, m))
    rows = _distinct_rows(counts, m, rng)
    vals = rng.standard_normal(rows.size)
    row_factor = rng.uniform(0.1, 10.0, size=m)
    return _csr_pair_from_columns(m, n, counts, rows, vals * row_factor[rows])


def general_cfg2(seed: int = 0) -> LP:
    """The power-law workload's shape (100,000 x 400,000, ~3.2M nonzeros) in
    general form."""
    rng = rng_for(13, seed)
    A, AT = _cfg2_matrix(100_000, 400_000, rng, 2000)
    return general_from_matrix(A, AT, rng, name=f"gcfg2_s{seed}", meta={"cfg": 2, "seed": seed})


def general_cfg2_sub(seed: int = 0, scale: int = 100) -> LP:
    rng = rng_for(13, 1000 + scale, seed)
    A, AT = _cfg2_matrix(100_000 // scale, 400_000 // scale, rng, 2000)
    return general_from_matrix(A, AT, rng, name=f"gcfg2sub{scale}_s{seed}",
                               meta={"cfg": 2, "seed": seed, "scale": scale})


# ---------------------------------------------------------------------------
# LPs without an optimum (no planted point: x_star, y_star, z_star are None)
# ---------------------------------------------------------------------------

def _lp_from_dense(A: np.ndarray, b, c, name: str, lo=None, hi=None, sense=None) -> LP:
    Acsr = sp.csr_matrix(np.asarray(A, dtype=np.float64))
    Acsr.sort_indices()
    AT = sp.csr_matrix(Acsr.T)
    AT.sort_indices()
    for M in (Acsr, AT):
        M.indices = M.indices.astype(np.int32)
        M.indptr = M.indptr.astype(np.int32)
    return LP(Acsr, AT, np.asarray(b, dtype=np.float64), np.asarray(c, dtype=np.float64), None, None, None,
              name=name, lo=lo, hi=hi, sense=sense)


def farkas_tiny() -> LP:
    """x1 + x2 = -1, x >= 0: infeasible (y = -1 is a Farkas ray)."""
    return _lp_from_dense([[1.0, 1.0]], [-1.0], [1.0, 1.0], "farkas_tiny")


def unbounded_tiny() -> LP:
    """min -x1 s.t. x1 - x2 = 0, x >= 0: unbounded along (1, 1)."""
    return _lp_from_dense([[1.0, -1.0]], [0.0], [-1.0, 0.0], "unbounded_tiny")


def conflicting_rows(seed: int) -> LP:
    """A general tiny LP plus two copies of its first row's coefficients, one
    >= 1 and one <= 0: infeasible."""
    g = general_tiny(10, 24, 3, 200 + seed)
    A = sp.vstack([g.A, g.A[0], g.A[0]]).toarray()
    return _lp_from_dense(A, np.concatenate([g.b, [1.0, 0.0]]), g.c, f"conflict_s{seed}", g.lo, g.hi,
                          np.concatenate([g.sense, np.array([SENSE_GE, SENSE_LE], dtype=np.int8)]))


def unbounded_column(seed: int) -> LP:
    """A general tiny LP with an extra free column that is in no row and
    costs 1: unbounded below."""
    g = general_tiny(10, 24, 3, 300 + seed)
    A = np.hstack([g.A.toarray(), np.zeros((g.m, 1))])
    return _lp_from_dense(A, g.b, np.concatenate([g.c, [1.0]]), f"unbounded_s{seed}",
                          np.concatenate([g.lo, [-np.inf]]), np.concatenate([g.hi, [np.inf]]), g.sense)


def box_infeasible() -> LP:
    """x1 + x2 = 5 with both in [0, 1]: infeasible."""
    return _lp_from_dense([[1.0, 1.0]], [5.0], [1.0, -1.0], "box_infeasible", np.zeros(2), np.ones(2),
                          np.zeros(1, dtype=np.int8))
