// SpMV shape autotuner: times candidate shapes of the iteration kernels on the
// caller's own matrix (a short run of every candidate with per-kernel HIP
// events) and returns the fastest in the options.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mipdhg.h"

namespace mip {
void set_error(const char* fmt, ...);
int64_t tile_count(const std::vector<int32_t>& rowptr, int32_t nrows, int32_t tile_nnz, int32_t tile_rows);
int column_hash(const int32_t* col, int64_t nnz, uint64_t* scratch, hipStream_t stream, uint64_t* out);
}

namespace {

// A candidate: the shape of A's tiles (dual) and of A^T's (primal).
struct Cand {
    int32_t kind, tile_nnz, tile_rows, short_row, tile_nnz_at, tile_rows_at, short_row_at;
};

// the library's default tile shape, and how much faster (ratio) another
// shape must be to replace it
constexpr int32_t kDefNnz = 2048, kDefRows = 512, kDefShort = -1;
constexpr double kMargin = 1.03;

std::vector<Cand> candidates() {
    std::vector<Cand> c;
    c.push_back({1, 0, 0, 0, 0, 0, 0});  // lane groups with the planner's lane counts
    for (int kind : {0, 2})
        for (int tn : {1024, 2048, 4096, 8192})
            for (int tr : {256, 512})
                for (int sr : {-1, 32}) c.push_back({kind, tn, tr, sr, tn, tr, sr});
    // the dual on A's panel layout, which has no tile shape; its primal step
    // is kind 0's, so kind 0's fastest primal shape goes with it
    c.push_back({3, kDefNnz, kDefRows, kDefShort, kDefNnz, kDefRows, kDefShort});
    // (kind 4, both steps on panel layouts, is not a candidate: its layout
    // costs more setup than its primal saves on a solve of ordinary length)
    return c;
}

// The smallest tile size up to 2,048 nonzeros (8 products per thread) whose
// greedy cut gives at most `target` tiles of at most 512 rows (so the count
// is as close to the target as the cut allows), or 0 if none does.
int32_t balanced_nnz(const std::vector<int32_t>& rp, int32_t nrows, int64_t target) {
    int32_t lo = 256, hi = 2048;
    if (mip::tile_count(rp, nrows, hi, 512) > target) return 0;
    while (lo < hi) {  // the count does not grow with the tile size
        const int32_t mid = (lo + hi) / 2;
        if (mip::tile_count(rp, nrows, mid, 512) <= target) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// Tiles sized so that their count is a whole number k of workgroups per CU
// (k = 4..8): every CU then gets the same number of tiles of one wave.
void balanced_candidates(const mipdhg_lp* lp, hipStream_t s, std::vector<Cand>& out) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return;
    std::vector<int32_t> ra(lp->m + 1), rat(lp->n + 1);
    if (hipMemcpyAsync(ra.data(), lp->a_rowptr, ra.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(rat.data(), lp->at_rowptr, rat.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return;
    if (ra[0] != 0 || rat[0] != 0 || ra[lp->m] != lp->nnz || rat[lp->n] != lp->nnz) return;  // the solve reports it
    for (int k = 4; k <= 8; ++k) {
        const int32_t ta = balanced_nnz(ra, lp->m, (int64_t)k * cus);
        const int32_t tat = balanced_nnz(rat, lp->n, (int64_t)k * cus);
        if (ta > 0 && tat > 0)
            for (int sr : {-1, 32}) out.push_back({0, ta, 512, sr, tat, 512, sr});
    }
}

}  // namespace

extern "C" int mipdhg_autotune(const mipdhg_lp* lp, mipdhg_options* opt, int32_t iters, void* workspace,
                               size_t workspace_bytes, void* stream, double* x, double* y, double* z, double* r_p,
                               double* r_d, double* best_ms) {
    if (!lp || !opt || iters < 1) return mip::set_error("lp, opt and iters >= 1 are required"), MIPDHG_ERR_INVALID_ARG;
    // per spmv_kind: the fastest dual (A's tiles) and primal (A^T's tiles) shapes
    struct Best {
        double ms = 1e300;
        Cand c{0, 0, 0, 0, 0, 0, 0};
    };
    constexpr int kKinds = 5;
    Best dual[kKinds], primal[kKinds], dual_def[kKinds], primal_def[kKinds];
    bool first = true;
    const bool general = lp->lo || lp->hi || lp->sense;  // runs on the tile kernels only
    std::vector<Cand> cands = candidates();
    balanced_candidates(lp, (hipStream_t)stream, cands);
    for (const Cand& c : cands) {
        if (general && c.kind == 1) continue;
        if ((opt->restart_avg || opt->step_rule == 1) && c.kind != 0) continue;  // one workgroup per tile only
        mipdhg_options o = *opt;
        o.spmv_kind = c.kind;
        o.tile_nnz = c.tile_nnz;
        o.tile_rows = c.tile_rows;
        o.short_row = c.short_row;
        o.tile_nnz_at = c.tile_nnz_at;
        o.tile_rows_at = c.tile_rows_at;
        o.short_row_at = c.short_row_at;
        o.kernel_timing = 2;  // 256 back-to-back launches of each kernel, timed by events around them
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
        if (c.tile_nnz == kDefNnz && c.tile_rows == kDefRows && c.short_row == kDefShort &&
            c.tile_nnz_at == kDefNnz) {
            dual_def[c.kind] = Best{info.ms_dual, c};
            primal_def[c.kind] = Best{info.ms_primal, c};
        }
    }
    // keep the default shape unless a candidate beats it by more than the
    // timing noise, so that the choice is stable from run to run
    for (int k = 0; k < kKinds; ++k) {
        if (dual_def[k].ms < 1e300 && dual[k].ms * kMargin >= dual_def[k].ms) dual[k] = dual_def[k];
        if (primal_def[k].ms < 1e300 && primal[k].ms * kMargin >= primal_def[k].ms) primal[k] = primal_def[k];
    }
    if (primal[3].ms < 1e300 && primal[0].ms < 1e300) primal[3] = primal[0];
    int kind = -1;
    double best = 1e300;
    for (int k = 0; k < kKinds; ++k) {
        if (dual[k].ms >= 1e300 || primal[k].ms >= 1e300) continue;
        const double t = dual[k].ms + primal[k].ms;
        if (t < best) {
            best = t;
            kind = k;
        }
    }
    if (kind < 0) return mip::set_error("no candidate shape could be timed"), MIPDHG_ERR_UNSUPPORTED;
    opt->spmv_kind = kind;
    // kinds 3 and 4 still run the power iteration and the evaluations on the
    // tiles: the shapes of kind 0's fastest dual (A) and, for kind 4, primal (A^T)
    const Cand& ac = ((kind == 3 || kind == 4) && dual[0].ms < 1e300) ? dual[0].c : dual[kind].c;
    const Cand& pc = (kind == 4 && primal[0].ms < 1e300) ? primal[0].c : primal[kind].c;
    opt->tile_nnz = ac.tile_nnz;
    opt->tile_rows = ac.tile_rows;
    opt->short_row = ac.short_row;
    opt->tile_nnz_at = pc.tile_nnz_at;
    opt->tile_rows_at = pc.tile_rows_at;
    opt->short_row_at = pc.short_row_at;
    if (best_ms) *best_ms = best;
    return 0;
}

namespace {

// The shape fields the tuner chooses, and their text form in the cache file.
struct Shape {
    int32_t v[7];
    double ms;
};

std::mutex g_tune_mu;
std::map<std::string, Shape> g_tuned;  // this process's choices by signature

uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

// What the choice depends on: the device (architecture, compute units), the
// options that change the kernels or the candidates, the sizes, and the
// sparsity structure (row pointers of A and A^T, column indices of both).
int signature(const mipdhg_lp* lp, const mipdhg_options* opt, void* ws, hipStream_t s, std::string* out) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return mip::set_error("could not query the device"), MIPDHG_ERR_HIP;
    std::vector<int32_t> ra(lp->m + 1), rat(lp->n + 1);
    if (hipMemcpyAsync(ra.data(), lp->a_rowptr, ra.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(rat.data(), lp->at_rowptr, rat.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return mip::set_error("could not read the row pointers"), MIPDHG_ERR_HIP;
    uint64_t ca = 0, cat = 0;
    int rc;
    if ((rc = mip::column_hash(lp->a_col, lp->nnz, (uint64_t*)ws, s, &ca))) return rc;
    if ((rc = mip::column_hash(lp->at_col, lp->nnz, (uint64_t*)ws, s, &cat))) return rc;
    char buf[512];
    snprintf(buf, sizeof(buf), "%s:%d:p%d:g%d%d%d:a%d:m%d:n%d:z%lld:%016llx:%016llx:%016llx:%016llx", prop.gcnArchName,
             prop.multiProcessorCount, opt->precision, lp->lo != nullptr, lp->hi != nullptr, lp->sense != nullptr,
             opt->restart_avg, lp->m, lp->n, (long long)lp->nnz,
             (unsigned long long)fnv1a(ra.data(), ra.size() * 4), (unsigned long long)fnv1a(rat.data(), rat.size() * 4),
             (unsigned long long)ca, (unsigned long long)cat);
    for (char* c = buf; *c; ++c)
        if (*c == ' ') *c = '_';
    *out = buf;
    return 0;
}

void apply_shape(const Shape& sh, mipdhg_options* opt) {
    opt->spmv_kind = sh.v[0];
    opt->tile_nnz = sh.v[1];
    opt->tile_rows = sh.v[2];
    opt->short_row = sh.v[3];
    opt->tile_nnz_at = sh.v[4];
    opt->tile_rows_at = sh.v[5];
    opt->short_row_at = sh.v[6];
}

bool find_in_file(const char* path, const std::string& key, Shape* sh) {
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (fgets(line, sizeof(line), f)) {  // the last entry of a signature wins
        char k[600];
        Shape t;
        if (sscanf(line, "%599s %d %d %d %d %d %d %d %lf", k, &t.v[0], &t.v[1], &t.v[2], &t.v[3], &t.v[4], &t.v[5],
                   &t.v[6], &t.ms) == 9 &&
            key == k) {
            *sh = t;
            found = true;
        }
    }
    fclose(f);
    return found;
}

}  // namespace

extern "C" int mipdhg_autotune_cached(const mipdhg_lp* lp, mipdhg_options* opt, int32_t iters, const char* cache_path,
                                      void* workspace, size_t workspace_bytes, void* stream, double* x, double* y,
                                      double* z, double* r_p, double* r_d, double* best_ms, int32_t* hit) {
    if (!lp || !opt || iters < 1 || !workspace || workspace_bytes < 8)
        return mip::set_error("lp, opt, a workspace and iters >= 1 are required"), MIPDHG_ERR_INVALID_ARG;
    if (lp->m < 1 || lp->n < 1 || lp->nnz < 0 || !lp->a_rowptr || !lp->at_rowptr || !lp->a_col || !lp->at_col)
        return mip::set_error("the LP's sizes and structure arrays are required"), MIPDHG_ERR_INVALID_ARG;
    if (hit) *hit = 0;
    std::string key;
    int rc = signature(lp, opt, workspace, (hipStream_t)stream, &key);
    if (rc) return rc;
    Shape sh;
    bool found = false;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            sh = it->second;
            found = true;
        } else if (cache_path && find_in_file(cache_path, key, &sh)) {
            g_tuned[key] = sh;
            found = true;
        }
    }
    if (found) {
        apply_shape(sh, opt);
        if (best_ms) *best_ms = sh.ms;
        if (hit) *hit = 1;
        return 0;
    }
    double ms = 0.0;
    rc = mipdhg_autotune(lp, opt, iters, workspace, workspace_bytes, stream, x, y, z, r_p, r_d, &ms);
    if (rc) return rc;
    sh = Shape{{opt->spmv_kind, opt->tile_nnz, opt->tile_rows, opt->short_row, opt->tile_nnz_at, opt->tile_rows_at,
                opt->short_row_at},
               ms};
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tuned[key] = sh;
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "%s %d %d %d %d %d %d %d %.6f\n", key.c_str(), sh.v[0], sh.v[1], sh.v[2], sh.v[3], sh.v[4],
                    sh.v[5], sh.v[6], sh.ms);
            fclose(f);
        }
    }
    if (best_ms) *best_ms = ms;
    return 0;
}
