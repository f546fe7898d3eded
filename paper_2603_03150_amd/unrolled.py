"""torch.autograd.Function over the unrolled PDHG map x_K(c, b).

Forward and backward are single calls into libmipdhg (mipdhg_unrolled_forward
/ mipdhg_unrolled_backward); this module only moves pointers.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from .solver import DeviceBatch, make_options


class UnrolledMap:
    """The map for one batch structure (A fixed), K iterations, checkpoints
    every ckpt_every iterations.  Call .apply(c, b) for an autograd-aware x_K."""

    def __init__(self, batch: DeviceBatch, K: int = 2000, ckpt_every: int = 100, precision: str = "fp32",
                 **opts):
        self.batch = batch
        self.K = int(K)
        self.ckpt = int(ckpt_every)
        self.opts = make_options(precision, **opts)
        self.precision = precision
        lib = _lib.load()
        nb = C.c_size_t(0)
        _lib.check(lib.mipdhg_unrolled_tape_size(C.byref(batch.struct()), C.byref(self.opts), self.K, self.ckpt,
                                                 C.byref(nb)))
        self.tape_bytes = int(nb.value)

    def _struct(self, c: torch.Tensor, b: torch.Tensor) -> _lib.BatchStruct:
        st = self.batch.struct()
        st.whole.c = c.data_ptr()
        st.whole.b = b.data_ptr()
        return st

    def forward_raw(self, c: torch.Tensor, b: torch.Tensor, tape: torch.Tensor | None = None,
                    replay: bool = False) -> tuple[torch.Tensor, torch.Tensor]:
        lib = _lib.load()
        dev = self.batch.lp.device
        c = c.detach().to(device=dev, dtype=torch.float64).contiguous()
        b = b.detach().to(device=dev, dtype=torch.float64).contiguous()
        if tape is None:
            tape = torch.empty(self.tape_bytes, dtype=torch.uint8, device=dev)
        xK = torch.empty(self.batch.lp.n, dtype=torch.float64, device=dev)
        st = self._struct(c, b)
        rc = lib.mipdhg_unrolled_forward(C.byref(st), C.byref(self.opts), self.K, self.ckpt, int(replay),
                                         tape.data_ptr(), tape.numel(),
                                         torch.cuda.current_stream(dev).cuda_stream, xK.data_ptr())
        _lib.check(rc)
        return xK, tape

    def schedule(self, tape: torch.Tensor, inst: int) -> tuple[list, list, list]:
        """mipdhg_unrolled_schedule: instance inst's restart iterations and the
        (tau, sigma) of its epochs, as the forward pass recorded them on tape."""
        lib = _lib.load()
        dev = self.batch.lp.device
        cap = self.K // max(1, int(self.opts.eval_every)) + 2
        restart_at = (C.c_int32 * cap)()
        taus, sigmas = (C.c_double * cap)(), (C.c_double * cap)()
        nr = C.c_int32(0)
        st = self.batch.struct()
        rc = lib.mipdhg_unrolled_schedule(C.byref(st), C.byref(self.opts), self.K, self.ckpt, tape.data_ptr(),
                                          tape.numel(), int(inst), torch.cuda.current_stream(dev).cuda_stream, cap,
                                          restart_at, taus, sigmas, C.byref(nr))
        _lib.check(rc)
        k = nr.value
        return list(restart_at[:k]), list(taus[:k + 1]), list(sigmas[:k + 1])

    def backward_raw(self, c: torch.Tensor, b: torch.Tensor, tape: torch.Tensor,
                     grad_xK: torch.Tensor) -> tuple[torch.Tensor, torch.Tensor]:
        lib = _lib.load()
        dev = self.batch.lp.device
        c = c.detach().to(device=dev, dtype=torch.float64).contiguous()
        b = b.detach().to(device=dev, dtype=torch.float64).contiguous()
        g = grad_xK.detach().to(device=dev, dtype=torch.float64).contiguous()
        gc = torch.empty(self.batch.lp.n, dtype=torch.float64, device=dev)
        gb = torch.empty(self.batch.lp.m, dtype=torch.float64, device=dev)
        st = self._struct(c, b)
        rc = lib.mipdhg_unrolled_backward(C.byref(st), C.byref(self.opts), self.K, self.ckpt, tape.data_ptr(),
                                          tape.numel(), g.data_ptr(), torch.cuda.current_stream(dev).cuda_stream,
                                          gc.data_ptr(), gb.data_ptr())
        _lib.check(rc)
        return gc, gb

    def apply(self, c: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
        return PDHGUnrolled.apply(c, b, self)


class PDHGUnrolled(torch.autograd.Function):
    """x_K = PDHGUnrolled.apply(c, b, umap); gradients flow to c and b."""

    @staticmethod
    def forward(ctx, c, b, umap: UnrolledMap):
        xK, tape = umap.forward_raw(c, b)
        ctx.umap = umap
        ctx.tape = tape
        ctx.save_for_backward(c.detach(), b.detach())
        return xK.to(c.dtype)

    @staticmethod
    def backward(ctx, grad_xK):
        c, b = ctx.saved_tensors
        gc, gb = ctx.umap.backward_raw(c, b, ctx.tape, grad_xK)
        return gc.to(c.dtype), gb.to(b.dtype), None
