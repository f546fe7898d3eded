// C-ABI odds and ends: defaults, status text, thread-local error message.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "mipdhg.h"

namespace mip {

static thread_local char g_err[1024] = {0};

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

}  // namespace mip

extern "C" void mipdhg_default_options(mipdhg_options* o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->precision = MIPDHG_FP64;
    o->ruiz_iters = 10;
    o->pock_chambolle = 1;
    o->power_iters = 100;
    o->eval_every = 64;
    o->step_safety = 0.95;
    o->reflect_rho = 1.0;
    o->halpern = 1;
    o->restarts = 1;
    o->beta_suff = 0.2;
    o->beta_nec = 0.8;
    o->beta_art = 0.36;
    o->pw_theta = 0.5;
    o->max_iter = 1000000;
    o->time_limit_s = 1e4;
    o->validate = 1;
    o->use_graph = 1;
    o->infeas_tol = 1e-8;
}

extern "C" const char* mipdhg_status_string(int code) {
    switch (code) {
        case MIPDHG_OPTIMAL: return "OPTIMAL";
        case MIPDHG_ITER_LIMIT: return "ITER_LIMIT";
        case MIPDHG_TIME_LIMIT: return "TIME_LIMIT";
        case MIPDHG_NUMERICAL: return "NUMERICAL";
        case MIPDHG_PRIMAL_INFEASIBLE: return "PRIMAL_INFEASIBLE";
        case MIPDHG_DUAL_INFEASIBLE: return "DUAL_INFEASIBLE";
        case MIPDHG_IN_PROGRESS: return "IN_PROGRESS";
        case MIPDHG_ERR_INVALID_ARG: return "ERR_INVALID_ARG";
        case MIPDHG_ERR_BAD_CSR: return "ERR_BAD_CSR";
        case MIPDHG_ERR_TRANSPOSE: return "ERR_TRANSPOSE";
        case MIPDHG_ERR_HIP: return "ERR_HIP";
        case MIPDHG_ERR_WORKSPACE: return "ERR_WORKSPACE";
        case MIPDHG_ERR_UNSUPPORTED: return "ERR_UNSUPPORTED";
        case MIPDHG_ERR_NONFINITE: return "ERR_NONFINITE";
        default: return "UNKNOWN";
    }
}

extern "C" const char* mipdhg_last_error(void) { return mip::g_err; }

extern "C" size_t mipdhg_sizeof(int which) {
    switch (which) {
        case 0: return sizeof(mipdhg_lp);
        case 1: return sizeof(mipdhg_options);
        case 2: return sizeof(mipdhg_info);
        case 3: return sizeof(mipdhg_batch);
        case 4: return sizeof(mipdhg_ipm_options);
        case 5: return sizeof(mipdhg_ipm_info);
        default: return 0;
    }
}
