"""Python face of the plain solve: device buffers from torch, then one C call.

Nothing here computes any part of the method; it allocates outputs and the
workspace with torch and passes raw device pointers and the current stream to
libmipdhg.
"""
from __future__ import annotations

import ctypes as C
from collections.abc import Sequence
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib


def _dev_tensor(a, dtype, device) -> torch.Tensor:
    t = torch.as_tensor(np.ascontiguousarray(a), dtype=dtype)
    return t.to(device)


class DeviceLP:
    """An LP held in device memory: A and A^T in CSR (int32 indices, float64
    values), b and c in float64; for the general form also the bounds lo, hi
    (float64, +-inf allowed) and the row senses (int8: 0 =, 1 >=, 2 <=), any
    of them None for its standard-form default (x >= 0, equality rows)."""

    def __init__(self, A, AT, b, c, device: str | torch.device = "cuda", lo=None, hi=None, sense=None):
        m, n = A.shape
        if AT.shape != (n, m):
            raise ValueError("AT must be n x m")
        self.m, self.n, self.nnz = int(m), int(n), int(A.nnz)
        self.device = torch.device(device)
        d = self.device
        self.a_rowptr = _dev_tensor(A.indptr, torch.int32, d)
        self.a_col = _dev_tensor(A.indices, torch.int32, d)
        self.a_val = _dev_tensor(A.data, torch.float64, d)
        self.at_rowptr = _dev_tensor(AT.indptr, torch.int32, d)
        self.at_col = _dev_tensor(AT.indices, torch.int32, d)
        self.at_val = _dev_tensor(AT.data, torch.float64, d)
        self.b = _dev_tensor(b, torch.float64, d)
        self.c = _dev_tensor(c, torch.float64, d)
        self.lo = None if lo is None else _dev_tensor(lo, torch.float64, d)
        self.hi = None if hi is None else _dev_tensor(hi, torch.float64, d)
        self.sense = None if sense is None else _dev_tensor(sense, torch.int8, d)

    @classmethod
    def from_lp(cls, lp, device="cuda") -> "DeviceLP":
        return cls(lp.A, lp.AT, lp.b, lp.c, device, getattr(lp, "lo", None), getattr(lp, "hi", None),
                   getattr(lp, "sense", None))

    def struct(self) -> _lib.LPStruct:
        s = _lib.LPStruct()
        s.m, s.n, s.nnz = self.m, self.n, self.nnz
        for name in ("a_rowptr", "a_col", "a_val", "at_rowptr", "at_col", "at_val", "b", "c"):
            setattr(s, name, getattr(self, name).data_ptr())
        for name in ("lo", "hi", "sense"):
            t = getattr(self, name)
            setattr(s, name, None if t is None else t.data_ptr())
        return s


def default_options() -> dict:
    lib = _lib.load()
    o = _lib.OptionsStruct()
    lib.mipdhg_default_options(C.byref(o))
    return {k: getattr(o, k) for k, _ in _lib.OptionsStruct._fields_
            if not k.startswith("trace_") and k not in ("x_init", "y_init")}


def make_options(precision: str = "fp64", **kw) -> _lib.OptionsStruct:
    lib = _lib.load()
    o = _lib.OptionsStruct()
    lib.mipdhg_default_options(C.byref(o))
    o.precision = _lib.PRECISION[precision]
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


@dataclass
class Solution:
    status: int
    status_name: str
    x: torch.Tensor
    y: torch.Tensor
    z: torch.Tensor
    r_p: torch.Tensor
    r_d: torch.Tensor
    d_row: torch.Tensor
    d_col: torch.Tensor
    info: dict
    trace: dict = field(default_factory=dict)
    workspace: torch.Tensor | None = None  # holds the state a resumed solve continues


def workspace_bytes(dlp: DeviceLP, precision: str = "fp64", **opts) -> int:
    lib = _lib.load()
    o = make_options(precision, **opts)
    nb = C.c_size_t(0)
    _lib.check(lib.mipdhg_workspace_size(C.byref(dlp.struct()), C.byref(o), C.byref(nb)))
    return int(nb.value)


def autotune(dlp: DeviceLP, precision: str = "fp32", iters: int = 128, cache: str | None = None, **opts) -> dict:
    """Pick the fastest SpMV shape for this LP (mipdhg_autotune_cached: a
    matrix structure seen before in this process, or listed in the file
    `cache`, is not timed again); returns the option fields to pass to
    solve(), plus 'cache_hit'."""
    lib = _lib.load()
    o = make_options(precision, **opts)
    need = 0
    for extra in (dict(tile_nnz=512, tile_rows=256), dict(spmv_kind=3)):  # smallest tiles; the panel layout
        need = max(need, workspace_bytes(dlp, precision, **dict(opts, **extra)))
    d = dlp.device
    ws = torch.empty(need, dtype=torch.uint8, device=d)
    f64 = dict(dtype=torch.float64, device=d)
    bufs = [torch.empty(k, **f64) for k in (dlp.n, dlp.m, dlp.n, dlp.m, dlp.n)]
    best = C.c_double(0.0)
    hit = C.c_int32(0)
    rc = lib.mipdhg_autotune_cached(C.byref(dlp.struct()), C.byref(o), int(iters),
                                    None if cache is None else str(cache).encode(), ws.data_ptr(), ws.numel(),
                                    torch.cuda.current_stream(d).cuda_stream, *[b.data_ptr() for b in bufs],
                                    C.byref(best), C.byref(hit))
    _lib.check(rc)
    return {"spmv_kind": o.spmv_kind, "tile_nnz": o.tile_nnz, "tile_rows": o.tile_rows, "short_row": o.short_row,
            "tile_nnz_at": o.tile_nnz_at, "tile_rows_at": o.tile_rows_at, "short_row_at": o.short_row_at,
            "ms_per_iter": best.value, "cache_hit": bool(hit.value)}


def solve(dlp: DeviceLP, eps: float = 1e-4, precision: str = "fp64", trace_iters: int = 0,
          x_init: torch.Tensor | None = None, y_init: torch.Tensor | None = None,
          workspace: torch.Tensor | None = None, resume: "Solution | torch.Tensor | None" = None,
          **opts) -> Solution:
    """Run mipdhg_solve on dlp.  Options are the fields of mipdhg_options.

    resume: a Solution of this LP, solved with the same options, whose state
    the solve continues (its workspace and output tensors are reused and
    written in place), or a workspace holding an imported state
    (import_state); max_iter counts all iterations."""
    lib = _lib.load()
    o = make_options(precision, **opts)
    resumed_ws = isinstance(resume, torch.Tensor)
    if resume is not None:
        o.resume = 1
        workspace = resume if resumed_ws else resume.workspace
    d = dlp.device
    f64 = dict(dtype=torch.float64, device=d)
    trace = {}
    if trace_iters:
        o.trace_iters = int(trace_iters)
        for key, size in (("x", dlp.n), ("y", dlp.m), ("xhat", dlp.n), ("yhat", dlp.m)):
            trace[key] = torch.zeros((trace_iters, size), **f64)
            setattr(o, "trace_" + key, trace[key].data_ptr())
    if x_init is not None:
        x_init = x_init.to(**f64).contiguous()
        o.x_init = x_init.data_ptr()
    if y_init is not None:
        y_init = y_init.to(**f64).contiguous()
        o.y_init = y_init.data_ptr()
    lps = dlp.struct()
    nb = C.c_size_t(0)
    _lib.check(lib.mipdhg_workspace_size(C.byref(lps), C.byref(o), C.byref(nb)))
    if resume is not None and (workspace is None or workspace.numel() < nb.value):
        raise ValueError("resume: the solution's workspace does not fit these options")
    if workspace is None or workspace.numel() < nb.value:
        workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=d)
    if resume is not None and not resumed_ws:
        x, y, z, r_p, r_d, d_row, d_col = (resume.x, resume.y, resume.z, resume.r_p, resume.r_d, resume.d_row,
                                           resume.d_col)
    else:
        x = torch.empty(dlp.n, **f64)
        y = torch.empty(dlp.m, **f64)
        z = torch.empty(dlp.n, **f64)
        r_p = torch.empty(dlp.m, **f64)
        r_d = torch.empty(dlp.n, **f64)
        d_row = torch.empty(dlp.m, **f64)
        d_col = torch.empty(dlp.n, **f64)
    info = _lib.InfoStruct()
    stream = torch.cuda.current_stream(d).cuda_stream
    rc = lib.mipdhg_solve(C.byref(lps), C.byref(o), float(eps), workspace.data_ptr(), workspace.numel(),
                          stream, x.data_ptr(), y.data_ptr(), z.data_ptr(), r_p.data_ptr(), r_d.data_ptr(),
                          d_row.data_ptr(), d_col.data_ptr(), C.byref(info))
    _lib.check(rc)
    return Solution(rc, lib.mipdhg_status_string(rc).decode(), x, y, z, r_p, r_d, d_row, d_col,
                    info.as_dict(), trace, workspace)


def state_bytes(dlp: DeviceLP, precision: str = "fp64", **opts) -> int:
    lib = _lib.load()
    o = make_options(precision, **opts)
    nb = C.c_size_t(0)
    _lib.check(lib.mipdhg_state_size(C.byref(dlp.struct()), C.byref(o), C.byref(nb)))
    return int(nb.value)


def export_state(dlp: DeviceLP, sol: Solution, precision: str = "fp64", **opts) -> torch.Tensor:
    """The resumable state of a solve (mipdhg_state_export) as a host uint8
    tensor; opts as for that solve."""
    lib = _lib.load()
    o = make_options(precision, **opts)
    out = torch.empty(state_bytes(dlp, precision, **opts), dtype=torch.uint8)
    _lib.check(lib.mipdhg_state_export(C.byref(dlp.struct()), C.byref(o), sol.workspace.data_ptr(),
                                       sol.workspace.numel(), out.data_ptr(), out.numel(),
                                       torch.cuda.current_stream(dlp.device).cuda_stream))
    return out


def import_state(dlp: DeviceLP, state: torch.Tensor, precision: str = "fp64", **opts) -> torch.Tensor:
    """A new workspace holding `state` (mipdhg_state_import), to pass as
    solve(..., resume=workspace) with the same options."""
    lib = _lib.load()
    o = make_options(precision, **opts)
    state = state.contiguous()
    ws = torch.empty(workspace_bytes(dlp, precision, **opts), dtype=torch.uint8, device=dlp.device)
    _lib.check(lib.mipdhg_state_import(C.byref(dlp.struct()), C.byref(o), ws.data_ptr(), ws.numel(),
                                       state.data_ptr(), state.numel(),
                                       torch.cuda.current_stream(dlp.device).cuda_stream))
    return ws


class DeviceBatch:
    """Independent LPs stacked block-diagonally in device memory, with the
    host offset arrays the batched entry point needs."""

    def __init__(self, A, AT, b, c, row_off, col_off, nnz_off, device="cuda"):
        self.lp = DeviceLP(A, AT, b, c, device)
        self.row_off = np.ascontiguousarray(row_off, dtype=np.int32)
        self.col_off = np.ascontiguousarray(col_off, dtype=np.int32)
        self.nnz_off = np.ascontiguousarray(nnz_off, dtype=np.int64)
        self.count = int(self.row_off.size - 1)

    @classmethod
    def from_lps(cls, lps, device="cuda") -> "DeviceBatch":
        """Stack LPs (objects with A, AT, b, c) into one block-diagonal pair."""
        import scipy.sparse as sp
        row_off = np.concatenate([[0], np.cumsum([lp.A.shape[0] for lp in lps])]).astype(np.int64)
        col_off = np.concatenate([[0], np.cumsum([lp.A.shape[1] for lp in lps])]).astype(np.int64)
        nnz_off = np.concatenate([[0], np.cumsum([lp.A.nnz for lp in lps])]).astype(np.int64)

        def stack(mats, off_minor, off_major):
            indptr = np.concatenate([mat.indptr[:-1].astype(np.int64) + nnz_off[i] for i, mat in enumerate(mats)]
                                    + [nnz_off[-1:]])
            indices = np.concatenate([mat.indices.astype(np.int64) + off_minor[i] for i, mat in enumerate(mats)])
            data = np.concatenate([mat.data for mat in mats])
            shape = (int(off_major[-1]), int(off_minor[-1]))
            return sp.csr_matrix((data, indices.astype(np.int32), indptr.astype(np.int32)), shape=shape)

        A = stack([lp.A for lp in lps], col_off, row_off)
        AT = stack([lp.AT for lp in lps], row_off, col_off)
        return cls(A, AT, np.concatenate([lp.b for lp in lps]), np.concatenate([lp.c for lp in lps]),
                   row_off, col_off, nnz_off, device)

    def struct(self) -> _lib.BatchStruct:
        s = _lib.BatchStruct()
        s.count = self.count
        s.row_off = self.row_off.ctypes.data
        s.col_off = self.col_off.ctypes.data
        s.nnz_off = self.nnz_off.ctypes.data
        s.whole = self.lp.struct()
        return s


@dataclass
class BatchSolution:
    status: int
    x: torch.Tensor
    y: torch.Tensor
    z: torch.Tensor
    r_p: torch.Tensor
    r_d: torch.Tensor
    infos: list
    workspace: torch.Tensor | None = None  # holds the state a resumed call continues

    def split(self, batch: DeviceBatch, i: int) -> dict:
        r0, r1 = batch.row_off[i], batch.row_off[i + 1]
        c0, c1 = batch.col_off[i], batch.col_off[i + 1]
        return {"x": self.x[c0:c1], "y": self.y[r0:r1], "z": self.z[c0:c1], "r_p": self.r_p[r0:r1],
                "r_d": self.r_d[c0:c1], "info": self.infos[i]}


def solve_batched(batch: DeviceBatch, eps=1e-4, precision: str = "fp32",
                  workspace: torch.Tensor | None = None, resume: "BatchSolution | None" = None,
                  **opts) -> BatchSolution:
    """Run mipdhg_solve_batched on every instance of the batch; eps is one
    tolerance for all instances or a sequence of one per instance.

    resume: the BatchSolution of an earlier call on this batch with the same
    options (batch_block_iters > 0) whose instances in progress this call
    continues; its workspace and output tensors are reused and written in
    place."""
    lib = _lib.load()
    o = make_options(precision, **opts)
    st = batch.struct()
    nb = C.c_size_t(0)
    _lib.check(lib.mipdhg_batch_workspace_size(C.byref(st), C.byref(o), C.byref(nb)))
    d = batch.lp.device
    f64 = dict(dtype=torch.float64, device=d)
    m, n = batch.lp.m, batch.lp.n
    if resume is not None:
        if not isinstance(resume, BatchSolution):
            raise TypeError("resume takes the BatchSolution of an earlier call")
        o.resume = 1
        workspace = resume.workspace
        if workspace is None or workspace.numel() < nb.value:
            raise ValueError("resume: the solution's workspace does not fit these options")
        x, y, z, r_p, r_d = resume.x, resume.y, resume.z, resume.r_p, resume.r_d
    else:
        if workspace is None or workspace.numel() < nb.value:
            workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=d)
        x, y, z = torch.empty(n, **f64), torch.empty(m, **f64), torch.empty(n, **f64)
        r_p, r_d = torch.empty(m, **f64), torch.empty(n, **f64)
    infos = (_lib.InfoStruct * batch.count)()
    stream = torch.cuda.current_stream(d).cuda_stream
    eps_arr = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), (batch.count,)))
    rc = lib.mipdhg_solve_batched(C.byref(st), C.byref(o), eps_arr.ctypes.data, workspace.data_ptr(), workspace.numel(),
                                  stream, x.data_ptr(), y.data_ptr(), z.data_ptr(), r_p.data_ptr(),
                                  r_d.data_ptr(), infos)
    _lib.check(rc)
    return BatchSolution(rc, x, y, z, r_p, r_d, _InfoList(infos), workspace)


class _InfoList(Sequence):
    """The per-instance reports as dicts, converted when read (a batch holds
    thousands; converting all of them costs milliseconds)."""

    def __init__(self, raw):
        self._raw = raw

    def __len__(self) -> int:
        return len(self._raw)

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self._raw[k].as_dict() for k in range(*i.indices(len(self._raw)))]
        if i < 0:
            i += len(self._raw)
        if not 0 <= i < len(self._raw):
            raise IndexError(i)
        return self._raw[i].as_dict()


def autotune_batched(batch: DeviceBatch, eps=1e-4, precision: str = "fp32", **opts) -> dict:
    """mipdhg_autotune_batched: the fastest batch_split for this batch (one
    timed batched solve per candidate); returns the option and its time."""
    lib = _lib.load()
    o = make_options(precision, **opts)
    st = batch.struct()
    nb = C.c_size_t(0)
    _lib.check(lib.mipdhg_batch_workspace_size(C.byref(st), C.byref(o), C.byref(nb)))
    d = batch.lp.device
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device=d)
    f64 = dict(dtype=torch.float64, device=d)
    m, n = batch.lp.m, batch.lp.n
    bufs = [torch.empty(k, **f64) for k in (n, m, n, m, n)]
    eps_arr = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), (batch.count,)))
    best = C.c_double(0.0)
    _lib.check(lib.mipdhg_autotune_batched(C.byref(st), C.byref(o), eps_arr.ctypes.data, ws.data_ptr(), ws.numel(),
                                           torch.cuda.current_stream(d).cuda_stream, *[b.data_ptr() for b in bufs],
                                           C.byref(best)))
    return {"batch_split": o.batch_split, "ms": best.value}


def batch_workspace_bytes(batch: DeviceBatch, precision: str = "fp32", **opts) -> int:
    lib = _lib.load()
    o = make_options(precision, **opts)
    nb = C.c_size_t(0)
    _lib.check(lib.mipdhg_batch_workspace_size(C.byref(batch.struct()), C.byref(o), C.byref(nb)))
    return int(nb.value)


def center_start(x: torch.Tensor, z: torch.Tensor, d_col: torch.Tensor | None = None, mu_min: float = 1e-6,
                 delta_max: float = 1e-4, alpha_min: float = 1e-6):
    """Algorithm 1's centered start (x', z', mu_target) from a PDHG solution;
    pass d_col to scale an original-space (x, z) first."""
    lib = _lib.load()
    n = int(x.numel())
    d = x.device
    x = x.to(torch.float64).contiguous()
    z = z.to(torch.float64).contiguous()
    ws = torch.empty(int(lib.mipdhg_center_workspace_size(n)), dtype=torch.uint8, device=d)
    xo = torch.empty(n, dtype=torch.float64, device=d)
    zo = torch.empty(n, dtype=torch.float64, device=d)
    mu = C.c_double(0.0)
    dc = d_col.to(torch.float64).contiguous() if d_col is not None else None
    rc = lib.mipdhg_center_start(n, x.data_ptr(), z.data_ptr(), dc.data_ptr() if dc is not None else None,
                                 mu_min, delta_max, alpha_min, ws.data_ptr(), ws.numel(),
                                 torch.cuda.current_stream(d).cuda_stream, xo.data_ptr(), zo.data_ptr(),
                                 C.byref(mu))
    _lib.check(rc)
    return xo, zo, mu.value


def center_reclamp(xp: torch.Tensor, zp: torch.Tensor, alpha_min: float) -> None:
    """In-place lift of both vectors to alpha_min (Algorithm 1 recovery loop)."""
    lib = _lib.load()
    _lib.check(lib.mipdhg_center_reclamp(int(xp.numel()), float(alpha_min),
                                         torch.cuda.current_stream(xp.device).cuda_stream,
                                         xp.data_ptr(), zp.data_ptr()))


def read_probe(buf: torch.Tensor, blocks: int = 2048) -> torch.Tensor:
    """Stream-read all of buf (a contiguous device tensor whose size is a
    multiple of 16 bytes) on the current stream (mipdhg_read_probe); returns
    the per-wave XOR words, asynchronously."""
    lib = _lib.load()
    if not buf.is_contiguous():
        raise ValueError("read_probe needs a contiguous tensor")
    out = torch.empty(blocks * 4, dtype=torch.int32, device=buf.device)
    _lib.check(lib.mipdhg_read_probe(buf.data_ptr(), buf.numel() * buf.element_size(), int(blocks),
                                     torch.cuda.current_stream(buf.device).cuda_stream, out.data_ptr()))
    return out


@dataclass
class IpmSolution:
    status: int
    status_name: str
    x: torch.Tensor
    y: torch.Tensor
    z: torch.Tensor
    info: dict


def ipm_options(**kw) -> _lib.IpmOptionsStruct:
    lib = _lib.load()
    o = _lib.IpmOptionsStruct()
    lib.mipdhg_ipm_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown interior-point option {k}")
        setattr(o, k, v)
    return o


def _ipm_call(dlp: DeviceLP, fn: str, d_row, d_col, point, **opts) -> IpmSolution:
    lib = _lib.load()
    o = ipm_options(**opts)
    lps = dlp.struct()
    nb = C.c_size_t(0)
    _lib.check(lib.mipdhg_ipm_workspace_size(C.byref(lps), C.byref(nb)))
    d = dlp.device
    f64 = dict(dtype=torch.float64, device=d)
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device=d)
    x, y, z = torch.empty(dlp.n, **f64), torch.empty(dlp.m, **f64), torch.empty(dlp.n, **f64)
    keep = [None if v is None else v.to(**f64).contiguous() for v in (d_row, d_col, *point)]
    ptr = [None if v is None else v.data_ptr() for v in keep]
    info = _lib.IpmInfoStruct()
    rc = getattr(lib, fn)(C.byref(lps), *ptr, C.byref(o), ws.data_ptr(), ws.numel(),
                          torch.cuda.current_stream(d).cuda_stream, x.data_ptr(), y.data_ptr(), z.data_ptr(),
                          C.byref(info))
    _lib.check(rc)
    return IpmSolution(rc, lib.mipdhg_status_string(rc).decode(), x, y, z, info.as_dict())


def ipm_solve(dlp: DeviceLP, d_row=None, d_col=None, start=None, **opts) -> IpmSolution:
    """mipdhg_ipm_solve: the interior-point method on the LP scaled by
    (d_row, d_col) (None: unscaled), from the scaled-space point
    start = (x, y, z), or from Mehrotra's point when start is None."""
    return _ipm_call(dlp, "mipdhg_ipm_solve", d_row, d_col, start if start is not None else (None, None, None),
                     **opts)


def ipm_warm(dlp: DeviceLP, sol: "Solution", **opts) -> IpmSolution:
    """mipdhg_ipm_warm: Algorithm 1 from a PDHG solution of dlp (its x, y, z
    and scaling), then the interior-point method with the alpha_min loop."""
    return _ipm_call(dlp, "mipdhg_ipm_warm", sol.d_row, sol.d_col, (sol.x, sol.y, sol.z), **opts)
