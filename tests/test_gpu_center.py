"""GPU Algorithm 1 (Section 3.1) against the oracle's element-by-element map."""
import numpy as np
import pytest

import lpgen
import oracle
from oracle.centering import center, reclamp

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_03150_amd")
torch = pytest.importorskip("torch")


def test_center_matches_oracle_on_random_pairs():
    rng = np.random.default_rng(8)
    n = 100_003
    x = np.where(rng.random(n) < 0.5, 0.0, rng.exponential(1.0, n))
    z = np.where(x > 0, rng.exponential(1e-3, n) * (rng.random(n) < 0.2), rng.exponential(1.0, n))
    xo, zo, mu = P.center_start(torch.tensor(x, device="cuda"), torch.tensor(z, device="cuda"))
    rx, rz, rmu = center(x, z)
    assert abs(mu - rmu) <= 1e-14 * rmu
    assert np.allclose(xo.cpu().numpy(), rx, rtol=1e-13, atol=0)
    assert np.allclose(zo.cpu().numpy(), rz, rtol=1e-13, atol=0)
    a, b = reclamp(rx, rz, 1e-5)
    P.center_reclamp(xo, zo, 1e-5)
    assert np.allclose(xo.cpu().numpy(), a, rtol=1e-13) and np.allclose(zo.cpu().numpy(), b, rtol=1e-13)


def test_center_from_solve_output_scales_first():
    lp = lpgen.cfg1(0)
    sol = P.solve(P.DeviceLP.from_lp(lp), 1e-4, "fp64")
    xo, zo, mu = P.center_start(sol.x, sol.z, d_col=sol.d_col)
    dc = sol.d_col.cpu().numpy()
    rx, rz, rmu = center(sol.x.cpu().numpy() / dc, sol.z.cpu().numpy() * dc)
    assert abs(mu - rmu) <= 1e-14 * rmu
    assert np.allclose(xo.cpu().numpy(), rx, rtol=1e-13) and np.allclose(zo.cpu().numpy(), rz, rtol=1e-13)
    assert (xo > 0).all() and (zo > 0).all()
