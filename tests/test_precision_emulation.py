"""Why the GPU's reduced-precision iteration holds its iterates relative to
the epoch's anchor (CPU emulation, tests/emul_precision.py).

Float64: both storage layouts are the oracle's iteration (same status,
iteration count and objective).  Float32, on a power-law LP at 1e-6: with
the iterates, b~ and c~ stored directly, the rounded values make the scaled
LP drift (its optimal face has recession directions, and a perturbation of
the data gives some of them a descent slope); x grows and the run never
reaches 1e-6.  Stored relative to the anchor, with the anchor's residuals
formed in float64 at each restart, every rounding error scales with the
epoch's movement and the run reaches 1e-6 with the objective of the planted
optimum.
"""
import numpy as np
import pytest

import emul_precision as emu
import lpgen
import oracle


@pytest.mark.parametrize("layout", ["direct", "anchor"])
def test_float64_layouts_are_the_oracle_iteration(layout):
    lp = lpgen.cfg1(1)
    ref = oracle.solve(lp.A, lp.AT, lp.b, lp.c, 1e-7)
    st, it, me, _ = emu.run(lp.A, lp.AT, lp.b, lp.c, 1e-7, layout, 100_000, rnd=lambda a: a)
    assert (st, it) == (ref.status, ref.iters)
    assert abs(me.pobj - ref.meas.pobj) <= 1e-9 * abs(ref.meas.pobj)
    assert np.abs(me.x - ref.meas.x).max() <= 1e-9 * max(1.0, np.abs(ref.meas.x).max())


def test_float32_storage_relative_to_the_anchor_reaches_1e6():
    lp = lpgen.cfg2_sub(0, scale=25)
    st_a, it_a, me_a, _ = emu.run(lp.A, lp.AT, lp.b, lp.c, 1e-6, "anchor", 2560)
    st_d, it_d, me_d, _ = emu.run(lp.A, lp.AT, lp.b, lp.c, 1e-6, "direct", 2560)
    assert st_a == 0 and it_a <= 2560
    assert abs(me_a.pobj - lp.p_star) <= 1e-5 * abs(lp.p_star)
    nb = np.linalg.norm(lp.b)
    assert st_d == 1 and me_d.rp_norm > 1e-4 * (1 + nb)  # still 100x off after as many iterations
