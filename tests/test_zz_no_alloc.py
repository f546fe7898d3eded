"""The allocation-free centring entry point against the workspace one.

mipdhg_center_start_noalloc keeps its scratch in a device array of the
library instead of a caller workspace.  Called through the C ABI twice in a
row (the second call smaller, so that it runs on what the first left in the
scratch), its outputs and target must equal those of mipdhg_center_start on
the same inputs bit for bit: both run the same kernels in the same order.
"""
import ctypes as C

import numpy as np
import pytest

from oracle.centering import center

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_03150_amd")
torch = pytest.importorskip("torch")
from paper_2603_03150_amd import _lib  # noqa: E402


def _pairs(n, seed):
    rng = np.random.default_rng(seed)
    x = np.where(rng.random(n) < 0.5, 0.0, rng.exponential(1.0, n))
    z = np.where(x > 0, rng.exponential(1e-3, n) * (rng.random(n) < 0.2), rng.exponential(1.0, n))
    d = rng.uniform(0.5, 2.0, n)
    return x, z, d


def _with_workspace(lib, x, z, d, stream):
    n = x.numel()
    ws = torch.empty(int(lib.mipdhg_center_workspace_size(n)), dtype=torch.uint8, device="cuda")
    xo, zo = torch.empty_like(x), torch.empty_like(z)
    mu = C.c_double(0.0)
    _lib.check(lib.mipdhg_center_start(n, x.data_ptr(), z.data_ptr(), d.data_ptr(), 1e-6, 1e-4, 1e-6,
                                       ws.data_ptr(), ws.numel(), stream, xo.data_ptr(), zo.data_ptr(),
                                       C.byref(mu)))
    return xo, zo, mu.value


def _no_alloc(lib, x, z, d, stream):
    n = x.numel()
    xo, zo = torch.empty_like(x), torch.empty_like(z)
    mu = C.c_double(0.0)
    _lib.check(lib.mipdhg_center_start_noalloc(n, x.data_ptr(), z.data_ptr(), d.data_ptr(), 1e-6, 1e-4, 1e-6,
                                               stream, xo.data_ptr(), zo.data_ptr(), C.byref(mu)))
    return xo, zo, mu.value


def test_no_alloc_equals_workspace_entry_point_on_two_calls():
    lib = _lib.load()
    stream = torch.cuda.current_stream().cuda_stream
    for n, seed in ((1_500_007, 1), (40_001, 2)):  # the second smaller than the first
        x, z, d = (torch.tensor(v, device="cuda") for v in _pairs(n, seed))
        a = _no_alloc(lib, x, z, d, stream)
        b = _with_workspace(lib, x, z, d, stream)
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and a[2] == b[2], n
        # and the map itself, against the oracle's
        dn = d.cpu().numpy()
        rx, rz, rmu = center(x.cpu().numpy() / dn, z.cpu().numpy() * dn)
        assert abs(a[2] - rmu) <= 1e-14 * rmu
        assert np.allclose(a[0].cpu().numpy(), rx, rtol=1e-13, atol=0)
        assert np.allclose(a[1].cpu().numpy(), rz, rtol=1e-13, atol=0)


def test_no_alloc_refuses_more_than_its_scratch_holds():
    lib = _lib.load()
    nmax = int(lib.mipdhg_center_noalloc_max_n())
    assert nmax == 1 << 21
    x = torch.zeros(1, dtype=torch.float64, device="cuda")
    rc = lib.mipdhg_center_start_noalloc(nmax + 1, x.data_ptr(), x.data_ptr(), None, 1e-6, 1e-4, 1e-6,
                                         torch.cuda.current_stream().cuda_stream, x.data_ptr(), x.data_ptr(), None)
    assert rc == -1
    assert b"allocation-free scratch" in lib.mipdhg_last_error()
