// Device-resident control block of the single-LP solver.
#pragma once
#include <stdint.h>

namespace mip {

// Written by the setup code and by the decide kernel at the end of every
// block of iterations; read (uniformly) by every iteration kernel.
struct Ctrl {
    // read by the iteration kernels
    double tau, sigma;
    int64_t k_base;  // iterations since the last restart, at the block start
    int64_t t_base;  // iterations done, at the block start
    int32_t status;  // -1 while running, else a MIPDHG_* status
    int32_t restart_now;
    // restart and primal-weight state
    double omega, eta, R0, R_prev, last_R;
    int32_t restarts, do_restarts;
    // constants
    double eps, b_norm, c_norm, beta_suff, beta_nec, beta_art, pw_theta;
    int64_t max_iter;
    // last evaluation (original model)
    double rp2, rd2, pobj, dobj, xz, rp_inf, rd_inf;
    int64_t eval_t;
};

}  // namespace mip
