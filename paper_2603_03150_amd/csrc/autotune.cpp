// SpMV shape autotuner: times candidate shapes of the iteration kernels on the
// caller's own matrix (a short run of every candidate with per-kernel HIP
// events) and returns the fastest in the options.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "mipdhg.h"

namespace mip {
void set_error(const char* fmt, ...);
}

namespace {

struct Cand {
    int32_t kind, tile_nnz, tile_rows, short_row;
};

std::vector<Cand> candidates() {
    std::vector<Cand> c;
    c.push_back({1, 0, 0, 0});  // lane groups with the planner's lane counts
    for (int kind : {0, 2})
        for (int tn : {1024, 2048, 4096, 8192})
            for (int tr : {256, 512})
                for (int sr : {-1, 32}) c.push_back({kind, tn, tr, sr});
    return c;
}

}  // namespace

extern "C" int mipdhg_autotune(const mipdhg_lp* lp, mipdhg_options* opt, int32_t iters, void* workspace,
                               size_t workspace_bytes, void* stream, double* x, double* y, double* z, double* r_p,
                               double* r_d, double* best_ms) {
    if (!lp || !opt || iters < 1) return mip::set_error("lp, opt and iters >= 1 are required"), MIPDHG_ERR_INVALID_ARG;
    double best = 1e300;
    Cand win{0, 0, 0, 0};
    bool first = true;
    const bool general = lp->lo || lp->hi || lp->sense;  // runs on the tile kernels only
    for (const Cand& c : candidates()) {
        if (general && c.kind == 1) continue;
        mipdhg_options o = *opt;
        o.spmv_kind = c.kind;
        o.tile_nnz = c.tile_nnz;
        o.tile_rows = c.tile_rows;
        o.short_row = c.short_row;
        o.kernel_timing = 1;
        o.max_iter = iters;
        o.trace_iters = 0;
        o.resume = 0;
        o.validate = first ? opt->validate : 0;
        size_t need = 0;
        if (mipdhg_workspace_size(lp, &o, &need) != 0 || need > workspace_bytes) continue;
        mipdhg_info info;
        const int rc = mipdhg_solve(lp, &o, 0.0, workspace, workspace_bytes, stream, x, y, z, r_p, r_d, nullptr,
                                    nullptr, &info);
        if (rc < 0) {
            if (first) return rc;  // the matrix itself is rejected
            continue;               // this shape is not available (e.g. LDS)
        }
        first = false;
        const double ms = info.ms_primal + info.ms_dual;
        if (ms > 0.0 && ms < best) {
            best = ms;
            win = c;
        }
    }
    if (best >= 1e300) return mip::set_error("no candidate shape could be timed"), MIPDHG_ERR_UNSUPPORTED;
    opt->spmv_kind = win.kind;
    opt->tile_nnz = win.tile_nnz;
    opt->tile_rows = win.tile_rows;
    opt->short_row = win.short_row;
    if (best_ms) *best_ms = best;
    return 0;
}
