"""CPU oracle for the restarted-PDHG hot path.  TEST INFRASTRUCTURE ONLY.

This package is the slow, plain, float64 reference that the GPU library is
checked against.  Only the test suite, the smoke check and the benchmark's CPU
baseline leg may import it; the product path (the HIP library and its Python
binding) never does, and this package imports nothing from the product.

Contents
  pdhg.py       scaling, step size, PDHG iteration, evaluation, restarts,
                the differentiable unrolled map and its reverse/tangent modes
  centering.py  the centered warm-start map of Algorithm 1
  ipm.py        the interior-point consumer of that start (Mehrotra's
                predictor-corrector on the scaled LP, dense direct solves)

Parity status of each function is stated in its module header.
"""
from .pdhg import (  # noqa: F401
    OracleOptions, Measures, Result, validate, scale, power_sigma, step_size,
    initial_weight, pdhg_operator, evaluate, terminated, restart_due, solve,
    unrolled_forward, unrolled_grad, unrolled_tangent, Schedule, STATUS,
    SENSE_EQ, SENSE_GE, SENSE_LE, validate_general, reduced_costs, ray_measures, infeasibility,
    primal_weight_update,
)
