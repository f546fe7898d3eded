"""CPU emulation of the GPU iteration's reduced-precision storage (test harness).

Not the oracle: the oracle is float64 throughout.  This harness runs the
oracle's own steps (scaling, step size, primal weight, evaluation, restart
rule) with the quantities the GPU stores rounded to float32 where the GPU
stores them, and the arithmetic in float64 as in the kernels, in one of two
layouts:

* ``direct``: the matrix values, the iterates x, y, x_bar, the anchors and
  b~, c~ are stored rounded, as the tile kernels did before they held their
  iterates relative to the anchor;
* ``anchor``: the matrix values, u = x - x0, v = y - y0, x_bar - x0, the
  anchors and the anchor residuals r_b = b~ - A~ x0, r_c = c~ - A~^T y0 are
  stored rounded, and r_b, r_c are formed in float64 with the unrounded
  matrix at every restart (the current kernels).

In exact arithmetic both are the oracle's iteration.  Rounded, the first
perturbs the LP itself (float32 values, float32 b~ and c~) and injects
rounding of the whole iterate every step; the second's rounding errors scale
with the epoch's movement, which vanishes as the iteration converges.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

import oracle.pdhg as op
from oracle.pdhg import OracleOptions


def f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def run(A, AT, b, c, eps: float, layout: str, max_iter: int, opts: OracleOptions | None = None,
        rnd=f32):
    """Returns (status, iterations, measures, norm of x at the end)."""
    o = opts or OracleOptions()
    A = sp.csr_matrix(A)
    AT = sp.csr_matrix(AT)
    m, n = A.shape
    nb, nc = float(np.linalg.norm(b)), float(np.linalg.norm(c))
    d_row, d_col, At = op.scale(A, o.ruiz_iters, o.pock_chambolle)
    AtT = sp.csr_matrix(At.T)
    Ar = At.copy()
    Ar.data = rnd(At.data)
    ArT = sp.csr_matrix(Ar.T)
    bt, ct = d_row * b, d_col * c
    s_hat, hist = op.power_sigma(Ar, o.power_iters)
    eta = op.step_size(s_hat, hist, o)
    omega = op.initial_weight(bt, ct)
    tau, sig = eta / omega, eta * omega
    rho = o.reflect_rho
    x0, y0 = np.zeros(n), np.zeros(m)
    if layout == "anchor":
        u, v = np.zeros(n), np.zeros(m)
        rb, rc = rnd(bt - At @ x0), rnd(ct - AtT @ y0)
    else:
        x, y = np.zeros(n), np.zeros(m)
        btr, ctr = rnd(bt), rnd(ct)
    k, t, R0, R_prev = 0, 0, math.nan, math.inf
    pid = [0.0, 0.0, 0]
    while True:
        t += 1
        w = (k + 1.0) / (k + 2.0) if o.halpern else 1.0
        if layout == "anchor":
            g = rc - ArT @ v
            dxh = np.maximum(u - tau * g, -x0)
            ub = rnd(2.0 * dxh - u)
            dyh = v + sig * (rb - Ar @ ub)
            R = math.sqrt(omega * float(np.sum((u - dxh) ** 2)) + float(np.sum((v - dyh) ** 2)) / omega)
            u_new, v_new = rnd(w * ((1 + rho) * dxh - rho * u)), rnd(w * ((1 + rho) * dyh - rho * v))
            xh, yh = x0 + dxh, y0 + dyh
        else:
            g = ctr - ArT @ y
            xh = np.maximum(x - tau * g, 0.0)
            xb = rnd(2.0 * xh - x)
            yh = y + sig * (btr - Ar @ xb)
            R = math.sqrt(omega * float(np.sum((x - xh) ** 2)) + float(np.sum((y - yh) ** 2)) / omega)
            x_new = rnd(w * ((1 + rho) * xh - rho * x) + (1 - w) * x0)
            y_new = rnd(w * ((1 + rho) * yh - rho * y) + (1 - w) * y0)
        if k == 0:
            R0 = R
        k += 1
        if t % o.eval_every == 0 or t == max_iter:
            me = op.evaluate(A, AT, b, c, d_row, d_col, xh, yh)
            if op.terminated(me, nb, nc, eps):
                return 0, t, me, float(np.linalg.norm(me.x))
            if t >= max_iter:
                return 1, t, me, float(np.linalg.norm(me.x))
            if op.restart_due(R, R0, R_prev, k, t, o):
                dx, dy = float(np.linalg.norm(xh - x0)), float(np.linalg.norm(yh - y0))
                if dx > 1e-10 and dy > 1e-10:
                    omega = op.primal_weight_update(omega, dx, dy, pid, o)
                    tau, sig = eta / omega, eta * omega
                x0, y0 = rnd(xh), rnd(yh)
                if layout == "anchor":
                    u_new, v_new = np.zeros(n), np.zeros(m)
                    rb, rc = rnd(bt - At @ x0), rnd(ct - AtT @ y0)
                else:
                    x_new, y_new = x0.copy(), y0.copy()
                k, R_prev = 0, math.inf
            else:
                R_prev = R
        if layout == "anchor":
            u, v = u_new, v_new
        else:
            x, y = x_new, y_new
