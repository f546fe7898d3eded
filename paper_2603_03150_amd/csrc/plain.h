// Device-resident control block of the single-LP solver.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "common.h"

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
    // resume: iterations of the last evaluated block, the problem and layout
    // the state belongs to, and whether the state is the solve's own
    int32_t last_nit, resumable;
    uint64_t fingerprint;
    // infeasibility certificates: whether a previous evaluated point is kept
    int32_t have_prev, pw_count;
    double infeas_tol;
    // primal weight as a PID controller: gains, integral, previous error
    double pw_ki, pw_kd, pw_int, pw_err;
    // the step setup computed (what a resumed solve must recompute), and the
    // adaptive step rule's last decision and rejection count
    double eta0;
    int32_t accepted, step_rule;
    int64_t rejected;
};

// shared host helpers (plain.hip, validate.hip)
int check_lp(const mipdhg_lp* lp);
int check_options(const mipdhg_options* o);
int check_rowptr(const std::vector<int32_t>& rp, int32_t nrows, int64_t nnz, const char* which);
// Checks column ranges, finiteness of A, A^T, b, c, and A^T against A by a
// dot-product test.  flags: 4 ints, partials: >= 2 * max tiles doubles, red: 4.
int validate_device(const mipdhg_lp& lp, const TilePlan& ta, const TilePlan& tat, int32_t* flags,
                    double* partials, double* red, hipStream_t stream);

// Batched and unrolled solves: validate_device() on the whole block-diagonal
// pair, then every entry of an instance's rows (of A and of A^T) checked to lie
// in that instance's columns (rows).  rpa, rpat: the row pointers on the host;
// tiles_a, tiles_at: 4 * blockdiag_tile_slots() ints each; row_off_dev,
// col_off_dev: the instance offsets on the device; flags: 4 ints; partials:
// blockdiag_tile_slots() + 16 doubles; red: 4 doubles.
int validate_blockdiag(const mipdhg_batch& bt, const std::vector<int32_t>& rpa, const std::vector<int32_t>& rpat,
                       int32_t* tiles_a, int32_t* tiles_at, const int32_t* row_off_dev, const int32_t* col_off_dev,
                       int32_t* flags, double* partials, double* red, hipStream_t stream);
int64_t blockdiag_tile_slots(int64_t m, int64_t n, int64_t nnz);

int32_t tile_nnz_of(const mipdhg_options& o);
int32_t tile_rows_of(const mipdhg_options& o);
int32_t short_row_of(const mipdhg_options& o);
int32_t tile_nnz_at_of(const mipdhg_options& o);   // A^T's tiles (default: A's)
int32_t tile_rows_at_of(const mipdhg_options& o);
int32_t short_row_at_of(const mipdhg_options& o);
inline bool has_bounds(const mipdhg_lp& lp) { return lp.lo || lp.hi; }  // general form, columns
inline bool has_sense(const mipdhg_lp& lp) { return lp.sense != nullptr; } // general form, rows
inline bool is_general(const mipdhg_lp& lp) { return has_bounds(lp) || has_sense(lp); }
int iter_kind(const mipdhg_options& o, int64_t m, int64_t n);         // effective spmv_kind
bool sorted_layout(const mipdhg_options& o, int64_t m, int64_t n);  // sorted tile layout of the iteration copies
TilePlan make_tile_plan(const int32_t* rowptr, const int32_t* desc, int32_t ntiles, int32_t nrows, int32_t tnz,
                        int32_t trows, int32_t srow);
int allow_validate_lds(int bytes);
// Order-independent hash of a device column index array (the matrix
// structure the autotuner's choice depends on); scratch: 8 device bytes.
int column_hash(const int32_t* col, int64_t nnz, uint64_t* scratch, hipStream_t stream, uint64_t* out);

inline int grid_for(int64_t n, int cap = 2048) {
    int64_t g = (n + kBlock - 1) / kBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

}  // namespace mip
