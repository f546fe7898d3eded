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

// the library's default tile shape, and how much faster (ratio) another
// shape must be to replace it
constexpr int32_t kDefNnz = 2048, kDefRows = 512, kDefShort = -1;
constexpr double kMargin = 1.03;

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
    // per spmv_kind: the fastest dual (A's tiles) and primal (A^T's tiles) shapes
    struct Best {
        double ms = 1e300;
        Cand c{0, 0, 0, 0};
    };
    Best dual[3], primal[3], dual_def[3], primal_def[3];
    bool first = true;
    const bool general = lp->lo || lp->hi || lp->sense;  // runs on the tile kernels only
    for (const Cand& c : candidates()) {
        if (general && c.kind == 1) continue;
        mipdhg_options o = *opt;
        o.spmv_kind = c.kind;
        o.tile_nnz = c.tile_nnz;
        o.tile_rows = c.tile_rows;
        o.short_row = c.short_row;
        o.tile_nnz_at = o.tile_rows_at = o.short_row_at = 0;  // the same shape on both sides
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
        if (info.ms_dual > 0.0 && info.ms_dual < dual[c.kind].ms) dual[c.kind] = Best{info.ms_dual, c};
        if (info.ms_primal > 0.0 && info.ms_primal < primal[c.kind].ms) primal[c.kind] = Best{info.ms_primal, c};
        if (c.tile_nnz == kDefNnz && c.tile_rows == kDefRows && c.short_row == kDefShort) {
            dual_def[c.kind] = Best{info.ms_dual, c};
            primal_def[c.kind] = Best{info.ms_primal, c};
        }
    }
    // keep the default shape unless a candidate beats it by more than the
    // timing noise, so that the choice is stable from run to run
    for (int k = 0; k < 3; ++k) {
        if (dual_def[k].ms < 1e300 && dual[k].ms * kMargin >= dual_def[k].ms) dual[k] = dual_def[k];
        if (primal_def[k].ms < 1e300 && primal[k].ms * kMargin >= primal_def[k].ms) primal[k] = primal_def[k];
    }
    int kind = -1;
    double best = 1e300;
    for (int k = 0; k < 3; ++k) {
        if (dual[k].ms >= 1e300 || primal[k].ms >= 1e300) continue;
        const double t = dual[k].ms + primal[k].ms;
        if (t < best) {
            best = t;
            kind = k;
        }
    }
    if (kind < 0) return mip::set_error("no candidate shape could be timed"), MIPDHG_ERR_UNSUPPORTED;
    opt->spmv_kind = kind;
    opt->tile_nnz = dual[kind].c.tile_nnz;
    opt->tile_rows = dual[kind].c.tile_rows;
    opt->short_row = dual[kind].c.short_row;
    opt->tile_nnz_at = primal[kind].c.tile_nnz;
    opt->tile_rows_at = primal[kind].c.tile_rows;
    opt->short_row_at = primal[kind].c.short_row;
    if (best_ms) *best_ms = best;
    return 0;
}
