// Many independent LPs in one persistent launch.
//
// The instances are the diagonal blocks of one block-diagonal CSR pair.  Each
// workgroup takes instances from an atomic queue (largest first) and runs the
// whole method of the single solve on its instance: scaling, power iteration,
// the PDHG iterations, float64 evaluations on the original block and the
// restart / primal-weight rule, with __syncthreads() as the only phase barrier.
// The dual iterate y and the extrapolated primal x_bar, the two vectors the
// SpMVs gather from, live in LDS; everything else stays in L2-resident global
// memory.  Each thread owns fixed rows and columns of its instance, and every
// reduction is a fixed-order workgroup reduction whose result every thread
// holds, so all threads take the same decisions without a broadcast and the
// results do not depend on which workgroup ran the instance.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.h"
#include "inst_common.h"
#include "plain.h"

namespace mip {

struct BInst {  // per-instance result, device side
    int32_t status, restarts;
    int64_t iters;
    double rp2, rd2, pobj, dobj, xz, rp_inf, rd_inf;
    double b_norm, c_norm, sigma_hat, eta, omega0, omega;
};

struct BState {  // an instance's solve state between resumable calls
    int64_t t, k;
    double omega, tau, sig, R0, R_prev;
    int32_t restarts, phase;  // phase: 1 suspended, 2 finished
};

template <typename T, typename V>
struct BArgs {
    int32_t B;
    int32_t lds_m, lds_n;
    const int32_t* order;
    const int32_t* row_off;
    const int32_t* col_off;
    const int32_t *a_rowptr, *a_col;
    const double* a_val;
    const int32_t *at_rowptr, *at_col;
    const double* at_val;
    const double *b, *c;
    V *a_vs, *at_vs;
    uint16_t *a_cl, *at_cl;  // instance-local columns of A, A^T
    // the state relative to the epoch's anchor (x0, y0): x holds u = x - x0
    // (y's v = y - y0 is in LDS), ct and bt the anchor's residuals
    // c~ - A~^T y0 and b~ - A~ x0
    T *x, *x0, *xhat, *ct, *y0, *yhat, *bt;
    double *d_row, *d_col, *pu, *pav;
    double *xo, *yo, *zo, *rpo, *rdo;
    BInst* info;
    BState* state;
    T* ysave;  // y of suspended instances
    int32_t* counter;
    const double* eps;  // per-instance eps_rel
    int32_t resume, block_iters;
    double step_safety, rho, beta_suff, beta_nec, beta_art, theta;
    int64_t max_iter;
    int32_t ruiz, pc, power_iters, eval_every, halpern, restarts;
};

template <typename T, typename V, typename Acc, int BS>
__device__ void solve_instance(const BArgs<T, V>& a, int inst, T* yL, T* xbL, double* sh) {
    const int tid = threadIdx.x;
    const int r0 = a.row_off[inst], r1 = a.row_off[inst + 1];
    const int c0 = a.col_off[inst], c1 = a.col_off[inst + 1];
    const int m = r1 - r0, n = c1 - c0;
    double nomax[1] = {0.0};
    BState& st = a.state[inst];
    // phase of this instance in the workspace: 0 fresh, 1 suspended at the
    // end of a block, 2 finished (read by every thread: uniform)
    const int phase = a.resume ? st.phase : 0;
    if (phase == 2) return;  // finished in an earlier call: its outputs and report stand
    const double eps = a.eps[inst];
    double eta, omega, tau, sig, tol_p, tol_d;
    int64_t k, t;
    double R0, R_prev;
    int restarts;
    if (phase == 0) {
        const InstMat M{a.a_rowptr, a.a_col, a.a_val, a.at_rowptr, a.at_col, a.at_val, a.b, a.c};
        const InstSetup su = inst_setup<T, V, BS>(M, r0, r1, c0, c1, a.d_row, a.d_col, a.pu, a.pav, a.a_vs,
                                                  a.at_vs, a.a_cl, a.at_cl, a.bt, a.ct, a.ruiz, a.pc,
                                                  a.power_iters, a.step_safety, xbL, yL, sh);
        // the report's set-up fields are written now, so that they do not
        // stay live (in registers) across the iterations
        if (tid == 0) {
            BInst& r = a.info[inst];
            r.b_norm = su.b_norm;
            r.c_norm = su.c_norm;
            r.sigma_hat = su.sigma_hat;
            r.eta = su.eta;
            r.omega0 = su.omega0;
        }
        eta = su.eta;
        omega = su.omega0;
        tau = eta / omega;
        sig = eta * omega;
        tol_p = eps * (1.0 + su.b_norm);
        tol_d = eps * (1.0 + su.c_norm);
        k = 0;
        t = 0;
        R0 = NAN;
        R_prev = INFINITY;
        restarts = 0;
        // initial point (0, 0)
        for (int j = tid; j < n; j += BS) {
            a.x[c0 + j] = (T)0;
            a.x0[c0 + j] = (T)0;
        }
        for (int i = tid; i < m; i += BS) {
            yL[i] = (T)0;
            a.y0[r0 + i] = (T)0;
        }
    } else {
        // resume: the scaled matrix, b~, c~, the scaling, x, the anchors and
        // the report's set-up fields are still in the workspace; y and the
        // scalars were saved when the block ended
        const BInst& r = a.info[inst];
        eta = r.eta;
        tol_p = eps * (1.0 + r.b_norm);
        tol_d = eps * (1.0 + r.c_norm);
        omega = st.omega;
        tau = st.tau;
        sig = st.sig;
        k = st.k;
        t = st.t;
        R0 = st.R0;
        R_prev = st.R_prev;
        restarts = st.restarts;
        for (int i = tid; i < m; i += BS) yL[i] = a.ysave[r0 + i];
    }
    __syncthreads();

    const double rho = a.rho, opr = 1.0 + a.rho;
    const int E = a.eval_every;
    const int64_t t_begin = t;
    bool suspended = false;
    int status = -1;
    while (status < 0) {
        ++t;
        const bool is_eval = (t % E == 0) || (t == a.max_iter);
        const bool first = (k == 0);
        const double w = a.halpern ? (double)(k + 1) / (double)(k + 2) : 1.0;
        double q[4] = {0.0, 0.0, 0.0, 0.0};
        // primal step over the columns (rows of A^T); float64 arithmetic,
        // stored in T.  The next row's bounds and vector entries are loaded
        // (branch-free, clamped to the last row) while this row is summed.
        int nb0 = 0, nb1 = 0;
        T nx = 0, nx0 = 0, nct = 0;
        if (n > 0) {
            const int g = c0 + min(tid, n - 1);
            nb0 = a.at_rowptr[g];
            nb1 = a.at_rowptr[g + 1];
            nx = a.x[g];
            nx0 = a.x0[g];
            nct = a.ct[g];
        }
        for (int j = tid; j < n; j += BS) {
            const int g = c0 + j;
            const int b0 = nb0, b1 = nb1;
            const double u = (double)nx, x0 = (double)nx0, rc = (double)nct;
            {
                const int gn = c0 + min(j + BS, n - 1);
                nb0 = a.at_rowptr[gn];
                nb1 = a.at_rowptr[gn + 1];
                nx = a.x[gn];
                nx0 = a.x0[gn];
                nct = a.ct[gn];
            }
            // u = x - x0, v = y - y0 (in LDS), rc = c~ - A~^T y0:
            // x_hat = x0 + max(u - tau (rc - A~^T v), -x0)
            const Acc s = row_dot4<Acc>(a.at_vs, a.at_cl, yL, b0, b1);
            double uh = u - tau * (rc - (double)s);
            uh = uh < -x0 ? -x0 : uh;
            xbL[j] = (T)(2.0 * uh - u);  // x_bar - x0
            a.x[g] = (T)(w * (opr * uh - rho * u));
            if (first || is_eval) {
                const double d = u - uh;
                q[0] += d * d;
            }
            if (is_eval) {
                q[1] += uh * uh;
                const double xh = x0 + uh;
                a.xhat[g] = (T)xh;
                a.xo[g] = a.d_col[g] * xh;
            }
        }
        __syncthreads();
        // dual step over the rows of A, with the same prefetch
        int mb0 = 0, mb1 = 0;
        T mbt = 0;
        if (m > 0) {
            const int g = r0 + min(tid, m - 1);
            mb0 = a.a_rowptr[g];
            mb1 = a.a_rowptr[g + 1];
            mbt = a.bt[g];
        }
        for (int i = tid; i < m; i += BS) {
            const int g = r0 + i;
            const int b0 = mb0, b1 = mb1;
            const double rb = (double)mbt;
            {
                const int gn = r0 + min(i + BS, m - 1);
                mb0 = a.a_rowptr[gn];
                mb1 = a.a_rowptr[gn + 1];
                mbt = a.bt[gn];
            }
            // rb = b~ - A~ x0: y_hat = y0 + v + sigma (rb - A~ (x_bar - x0))
            const Acc s = row_dot4<Acc>(a.a_vs, a.a_cl, xbL, b0, b1);
            const double v = (double)yL[i];
            const double vh = v + sig * (rb - (double)s);
            yL[i] = (T)(w * (opr * vh - rho * v));
            if (first || is_eval) {
                const double d = v - vh;
                q[2] += d * d;
            }
            if (is_eval) {
                q[3] += vh * vh;
                const double yh = (double)a.y0[g] + vh;
                a.yhat[g] = (T)yh;
                a.yo[g] = a.d_row[g] * yh;
            }
        }
        __syncthreads();
        if (!(first || is_eval)) {
            ++k;
            continue;
        }
        wg_reduce<4, 0, BS>(q, nomax, sh);
        if (first) R0 = sqrt(omega * q[0] + q[2] / omega);
        ++k;
        if (!is_eval) continue;
        const double R = sqrt(omega * q[0] + q[2] / omega);
        // evaluation on the original block, float64
        double ev[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, evm[2] = {0.0, 0.0};
        for (int i = tid; i < m; i += BS) {
            const int g = r0 + i;
            double s = 0.0;
            for (int kz = a.a_rowptr[g]; kz < a.a_rowptr[g + 1]; ++kz) s += a.a_val[kz] * a.xo[a.a_col[kz]];
            const double rp = a.b[g] - s;
            a.rpo[g] = rp;
            ev[0] += rp * rp;
            ev[1] += a.b[g] * a.yo[g];
            evm[0] = fmax(evm[0], fabs(rp));
        }
        for (int j = tid; j < n; j += BS) {
            const int g = c0 + j;
            double s = 0.0;
            for (int kz = a.at_rowptr[g]; kz < a.at_rowptr[g + 1]; ++kz) s += a.at_val[kz] * a.yo[a.at_col[kz]];
            const double gg = a.c[g] - s;
            const double z = gg > 0.0 ? gg : 0.0;
            const double rd = gg - z;
            a.zo[g] = z;
            a.rdo[g] = rd;
            const double xv = a.xo[g];
            ev[2] += rd * rd;
            ev[3] += a.c[g] * xv;
            ev[4] += xv * z;
            evm[1] = fmax(evm[1], fabs(rd));
        }
        wg_reduce<5, 2, BS>(ev, evm, sh);
        const double rp = sqrt(ev[0]), rd = sqrt(ev[2]), pobj = ev[3], dobj = ev[1];
        const double gap = fabs(pobj - dobj);
        if (!(isfinite(ev[0]) && isfinite(ev[2]) && isfinite(pobj) && isfinite(dobj))) status = MIPDHG_NUMERICAL;
        else if (rp <= tol_p && rd <= tol_d && gap <= eps * (1.0 + fabs(pobj) + fabs(dobj)))
            status = MIPDHG_OPTIMAL;
        else if (t >= a.max_iter) status = MIPDHG_ITER_LIMIT;
        if (tid == 0) {  // the latest evaluation's measures
            BInst& r = a.info[inst];
            r.rp2 = ev[0];
            r.rd2 = ev[2];
            r.pobj = ev[3];
            r.dobj = ev[1];
            r.xz = ev[4];
            r.rp_inf = evm[0];
            r.rd_inf = evm[1];
        }
        if (status >= 0) break;
        bool restart = false;
        if (a.restarts)
            restart = (R <= a.beta_suff * R0) || (R <= a.beta_nec * R0 && R > R_prev) ||
                      ((double)k >= a.beta_art * (double)t);
        if (restart) {
            const double dx = sqrt(q[1]), dy = sqrt(q[3]);
            if (dx > 1e-10 && dy > 1e-10) {
                omega = exp(a.theta * log(dy / dx) + (1.0 - a.theta) * log(omega));
                tau = eta / omega;
                sig = eta * omega;
            }
            // the anchor moves to (x_hat, y_hat), the state to 0, and the new
            // anchor's residuals are formed in float64 on the caller's
            // matrix: rb = D_r (b - A D_c x0), rc = D_c (c - A^T D_r y0)
            for (int j = tid; j < n; j += BS) {
                a.x0[c0 + j] = a.xhat[c0 + j];
                a.x[c0 + j] = (T)0;
            }
            for (int i = tid; i < m; i += BS) {
                a.y0[r0 + i] = a.yhat[r0 + i];
                yL[i] = (T)0;
            }
            __syncthreads();
            for (int i = tid; i < m; i += BS) {
                const int g = r0 + i;
                double sa = 0.0;
                for (int kz = a.a_rowptr[g]; kz < a.a_rowptr[g + 1]; ++kz) {
                    const int jc = a.a_col[kz];
                    sa += a.a_val[kz] * (a.d_col[jc] * (double)a.x0[jc]);
                }
                a.bt[g] = (T)(a.d_row[g] * (a.b[g] - sa));
            }
            for (int j = tid; j < n; j += BS) {
                const int g = c0 + j;
                double sa = 0.0;
                for (int kz = a.at_rowptr[g]; kz < a.at_rowptr[g + 1]; ++kz) {
                    const int ir = a.at_col[kz];
                    sa += a.at_val[kz] * (a.d_row[ir] * (double)a.y0[ir]);
                }
                a.ct[g] = (T)(a.d_col[g] * (a.c[g] - sa));
            }
            k = 0;
            R_prev = INFINITY;
            ++restarts;
            __syncthreads();
        } else {
            R_prev = R;
        }
        // end of this call's block: the state after an evaluation and its
        // restart decision is what the next iteration starts from
        if (a.block_iters > 0 && t - t_begin >= a.block_iters) {
            suspended = true;
            break;
        }
    }
    if (suspended) {
        for (int i = tid; i < m; i += BS) a.ysave[r0 + i] = yL[i];
        status = MIPDHG_IN_PROGRESS;
    }
    if (tid == 0) {
        st.phase = suspended ? 1 : 2;
        st.t = t;
        st.k = k;
        st.omega = omega;
        st.tau = tau;
        st.sig = sig;
        st.R0 = R0;
        st.R_prev = R_prev;
        st.restarts = restarts;
        BInst& r = a.info[inst];
        r.status = status;
        r.restarts = restarts;
        r.iters = t;
        r.omega = omega;
    }
    __syncthreads();
}

// Workgroup size of the split's launch of large instances: twice the
// threads on each instance's rows and columns.
constexpr int kBatchWide = 512;

template <typename T, typename V, typename Acc, int BS>
__global__ __launch_bounds__(BS) void k_batched(BArgs<T, V> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    T* yL = (T*)smem;
    T* xbL = yL + a.lds_m;
    __shared__ double sh[8 * (BS / kWave)];
    __shared__ int next;
    while (true) {
        if (threadIdx.x == 0) next = atomicAdd(a.counter, 1);
        __syncthreads();
        const int qi = __builtin_amdgcn_readfirstlane(next);  // uniform: scalar loads of the offsets
        __syncthreads();
        if (qi >= a.B) break;  // uniform: every wave leaves once the queue is empty
        solve_instance<T, V, Acc, BS>(a, a.order[qi], yL, xbL, sh);
    }
}

__global__ void k_zero_i32(int32_t* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// block-diagonal structure: every entry of instance i's rows lies in its columns
__global__ void k_check_blockdiag(const int32_t* rowptr, const int32_t* col, const int32_t* row_off,
                                  const int32_t* col_off, int B, int32_t nrows, int32_t* flags) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrows;
         r += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = B;  // instance: row_off[lo] <= r < row_off[lo+1]
        while (hi - lo > 1) {
            const int mid = (lo + hi) / 2;
            if (row_off[mid] <= r) lo = mid;
            else hi = mid;
        }
        const int c0 = col_off[lo], c1 = col_off[lo + 1];
        for (int k = rowptr[r]; k < rowptr[r + 1]; ++k)
            if (col[k] < c0 || col[k] >= c1) {
                atomicOr(flags, 8);
                break;
            }
    }
}

int validate_blockdiag(const mipdhg_batch& bt, const std::vector<int32_t>& rpa, const std::vector<int32_t>& rpat,
                       int32_t* tiles_a, int32_t* tiles_at, const int32_t* row_off_dev, const int32_t* col_off_dev,
                       int32_t* flags, double* partials, double* red, hipStream_t stream) {
    const mipdhg_lp& lp = bt.whole;
    const std::vector<int32_t> ta = make_tile_desc(rpa, lp.m, kTileNnzDefault, kTileRowsDefault),
                               tat = make_tile_desc(rpat, lp.n, kTileNnzDefault, kTileRowsDefault);
    if (!tile_desc_ok(ta, rpa, lp.m, kTileNnzDefault, kTileRowsDefault) ||
        !tile_desc_ok(tat, rpat, lp.n, kTileNnzDefault, kTileRowsDefault))
        return set_error("internal: tile plan does not cover the rows"), MIPDHG_ERR_UNSUPPORTED;
    MIP_HIP(hipMemcpyAsync(tiles_a, ta.data(), ta.size() * 4, hipMemcpyHostToDevice, stream));
    MIP_HIP(hipMemcpyAsync(tiles_at, tat.data(), tat.size() * 4, hipMemcpyHostToDevice, stream));
    const TilePlan pa = make_tile_plan(lp.a_rowptr, tiles_a, (int32_t)(ta.size() / 4), lp.m, kTileNnzDefault,
                                       kTileRowsDefault, kShortRowDefault);
    const TilePlan pat = make_tile_plan(lp.at_rowptr, tiles_at, (int32_t)(tat.size() / 4), lp.n, kTileNnzDefault,
                                        kTileRowsDefault, kShortRowDefault);
    int rc;
    if ((rc = allow_validate_lds((int)std::max(tile_lds_bytes(pa, 8), tile_lds_bytes(pat, 8))))) return rc;
    if ((rc = validate_device(lp, pa, pat, flags, partials, red, stream))) return rc;
    MIP_HIP(hipMemsetAsync(flags, 0, 4, stream));
    hipLaunchKernelGGL(k_check_blockdiag, dim3(grid_for(lp.m)), dim3(kBlock), 0, stream, lp.a_rowptr, lp.a_col,
                       row_off_dev, col_off_dev, bt.count, lp.m, flags);
    hipLaunchKernelGGL(k_check_blockdiag, dim3(grid_for(lp.n)), dim3(kBlock), 0, stream, lp.at_rowptr, lp.at_col,
                       col_off_dev, row_off_dev, bt.count, lp.n, flags);
    MIP_LAUNCH_CHECK();
    int32_t f = 0;
    MIP_HIP(hipMemcpyAsync(&f, flags, 4, hipMemcpyDeviceToHost, stream));
    MIP_HIP(hipStreamSynchronize(stream));
    if (f & 8) return set_error("an entry lies outside its instance's diagonal block"), MIPDHG_ERR_BAD_CSR;
    return 0;
}

int64_t blockdiag_tile_slots(int64_t m, int64_t n, int64_t nnz) {
    return std::max(max_tiles(m, nnz, kTileNnzDefault, kTileRowsDefault),
                    max_tiles(n, nnz, kTileNnzDefault, kTileRowsDefault));
}

struct BatchWs {
    uint64_t* hdr;  // {marker, fingerprint} of the state the workspace holds
    int32_t *order, *row_off, *col_off, *counter, *flags, *tiles_a, *tiles_at;
    BInst* info;
    BState* state;
    double *d_row, *d_col, *pu, *pav, *partials, *red, *eps;
    void *a_vs, *at_vs, *x, *x0, *xhat, *ct, *y0, *yhat, *bt, *ysave;
    uint16_t *a_cl, *at_cl;
    size_t bytes;
};

static BatchWs carve_batch(void* base, size_t cap, int64_t B, int64_t m, int64_t n, int64_t nnz, int prec) {
    Carver cv(base, cap);
    BatchWs w;
    const size_t vs = prec == MIPDHG_FP64 ? 8 : (prec == MIPDHG_FP32_BF16A ? 2 : 4);
    const size_t ts = prec == MIPDHG_FP64 ? 8 : 4;
    w.hdr = cv.take<uint64_t>(4);
    w.order = cv.take<int32_t>(B);
    w.row_off = cv.take<int32_t>(B + 1);
    w.col_off = cv.take<int32_t>(B + 1);
    w.counter = cv.take<int32_t>(64);
    w.flags = cv.take<int32_t>(64);
    w.tiles_a = cv.take<int32_t>(4 * max_tiles(m, nnz, kTileNnzDefault, kTileRowsDefault));
    w.tiles_at = cv.take<int32_t>(4 * max_tiles(n, nnz, kTileNnzDefault, kTileRowsDefault));
    w.info = cv.take<BInst>(B);
    w.state = cv.take<BState>(B);
    w.eps = cv.take<double>(B);
    w.d_row = cv.take<double>(m);
    w.d_col = cv.take<double>(n);
    w.pu = cv.take<double>(n);
    w.pav = cv.take<double>(m);
    w.partials = cv.take<double>((size_t)std::max(max_tiles(m, nnz, kTileNnzDefault, kTileRowsDefault), max_tiles(n, nnz, kTileNnzDefault, kTileRowsDefault)) + 16);
    w.red = cv.take<double>(16);
    w.a_vs = cv.take<char>(nnz * vs);
    w.at_vs = cv.take<char>(nnz * vs);
    w.a_cl = cv.take<uint16_t>(nnz);
    w.at_cl = cv.take<uint16_t>(nnz);
    w.x = cv.take<char>(n * ts);
    w.x0 = cv.take<char>(n * ts);
    w.xhat = cv.take<char>(n * ts);
    w.ct = cv.take<char>(n * ts);
    w.y0 = cv.take<char>(m * ts);
    w.yhat = cv.take<char>(m * ts);
    w.bt = cv.take<char>(m * ts);
    w.ysave = cv.take<char>(m * ts);
    w.bytes = (cv.off + 255) & ~size_t(255);
    return w;
}

// Identity of a batched solve's state in its workspace: the batch's sizes
// and offsets and every option the iterations depend on (not eps_rel,
// max_iter, batch_block_iters, validate or resume).  FNV-1a over the fields.
static uint64_t batch_fingerprint(const mipdhg_batch& bt, const mipdhg_options& o) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t nb) {
        const unsigned char* c = (const unsigned char*)p;
        for (size_t i = 0; i < nb; ++i) h = (h ^ c[i]) * 1099511628211ull;
    };
    const int64_t sz[4] = {bt.count, bt.whole.m, bt.whole.n, bt.whole.nnz};
    mix(sz, sizeof(sz));
    mix(bt.row_off, ((size_t)bt.count + 1) * sizeof(int32_t));
    mix(bt.col_off, ((size_t)bt.count + 1) * sizeof(int32_t));
    mix(bt.nnz_off, ((size_t)bt.count + 1) * sizeof(int64_t));
    const int32_t iv[8] = {o.precision, o.ruiz_iters, o.pock_chambolle, o.power_iters,
                           o.eval_every, o.halpern, o.restarts, o.batch_split};
    mix(iv, sizeof(iv));
    const double dv[6] = {o.step_safety, o.reflect_rho, o.beta_suff, o.beta_nec, o.beta_art, o.pw_theta};
    mix(dv, sizeof(dv));
    return h;
}

constexpr uint64_t kBatchStateMarker = 0x6d69706468672d62ull;

static int check_batch(const mipdhg_batch* bt) {
    if (!bt) return set_error("batch is NULL"), MIPDHG_ERR_INVALID_ARG;
    if (bt->count < 1) return set_error("batch count must be >= 1"), MIPDHG_ERR_INVALID_ARG;
    if (!bt->row_off || !bt->col_off || !bt->nnz_off)
        return set_error("row_off, col_off and nnz_off are required"), MIPDHG_ERR_INVALID_ARG;
    int rc = check_lp(&bt->whole);
    if (rc) return rc;
    const int B = bt->count;
    if (bt->row_off[0] != 0 || bt->col_off[0] != 0 || bt->nnz_off[0] != 0 || bt->row_off[B] != bt->whole.m ||
        bt->col_off[B] != bt->whole.n || bt->nnz_off[B] != bt->whole.nnz)
        return set_error("instance offsets must start at 0 and end at m, n, nnz"), MIPDHG_ERR_INVALID_ARG;
    for (int i = 0; i < B; ++i)
        if (bt->row_off[i + 1] <= bt->row_off[i] || bt->col_off[i + 1] <= bt->col_off[i] ||
            bt->nnz_off[i + 1] < bt->nnz_off[i])
            return set_error("instance %d is empty or its offsets decrease", i), MIPDHG_ERR_INVALID_ARG;
    return 0;
}

static int lds_bytes_for(int max_m, int max_n, size_t ts) {
    return (int)(((size_t)max_m + (size_t)max_n) * ts + 16);
}

template <typename T, typename V, typename Acc>
static int batched_impl(const mipdhg_batch& bt, const mipdhg_options& o, const double* eps, void* ws, size_t ws_bytes,
                        hipStream_t stream, double* x, double* y, double* z, double* r_p, double* r_d,
                        mipdhg_info* info) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    const mipdhg_lp& lp = bt.whole;
    const int B = bt.count;
    BatchWs w = carve_batch(ws, ws_bytes, B, lp.m, lp.n, lp.nnz, o.precision);
    if (w.bytes > ws_bytes)
        return set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, w.bytes), MIPDHG_ERR_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return set_error("workspace must be 256-byte aligned"), MIPDHG_ERR_INVALID_ARG;
    // a resume continues only the state of this batch under these options;
    // the header is invalid while a call runs and valid once it returns
    const uint64_t fp = batch_fingerprint(bt, o);
    uint64_t hdr_in[2] = {0, 0};
    const uint64_t hdr_running[2] = {0, 0}, hdr_done[2] = {kBatchStateMarker, fp};
    if (o.resume) {
        MIP_HIP(hipMemcpyAsync(hdr_in, w.hdr, sizeof(hdr_in), hipMemcpyDeviceToHost, stream));
        MIP_HIP(hipStreamSynchronize(stream));
        if (hdr_in[0] != kBatchStateMarker || hdr_in[1] != fp)
            return set_error("resume: the workspace does not hold the state of this batch with these options"),
                   MIPDHG_ERR_INVALID_ARG;
    }
    int max_m = 0, max_n = 0;
    for (int i = 0; i < B; ++i) {
        max_m = std::max(max_m, bt.row_off[i + 1] - bt.row_off[i]);
        max_n = std::max(max_n, bt.col_off[i + 1] - bt.col_off[i]);
    }
    const int lds = lds_bytes_for(max_m, max_n, sizeof(T));
    if (lds > 150 * 1024 || max_m > kInstMaxDim || max_n > kInstMaxDim)
        return set_error("largest instance needs %d bytes of LDS (limit 150 KiB): m + n too large", lds),
               MIPDHG_ERR_UNSUPPORTED;
    // host checks of the row pointers against the instance offsets
    std::vector<int32_t> rpa(lp.m + 1), rpat(lp.n + 1);
    MIP_HIP(hipMemcpyAsync(rpa.data(), lp.a_rowptr, (lp.m + 1) * 4, hipMemcpyDeviceToHost, stream));
    MIP_HIP(hipMemcpyAsync(rpat.data(), lp.at_rowptr, (lp.n + 1) * 4, hipMemcpyDeviceToHost, stream));
    MIP_HIP(hipStreamSynchronize(stream));
    int rc;
    if ((rc = check_rowptr(rpa, lp.m, lp.nnz, "A"))) return rc;
    if ((rc = check_rowptr(rpat, lp.n, lp.nnz, "A^T"))) return rc;
    for (int i = 0; i <= B; ++i)
        if (rpa[bt.row_off[i]] != bt.nnz_off[i] || rpat[bt.col_off[i]] != bt.nnz_off[i])
            return set_error("nnz_off does not match the row pointers at instance %d", i), MIPDHG_ERR_BAD_CSR;
    // largest instances first; with a split, the instances whose vectors
    // need more than batch_split bytes come first in the order array (the
    // wide launch), each class largest first
    std::vector<int32_t> order(B);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int p, int q) {
        return bt.nnz_off[p + 1] - bt.nnz_off[p] > bt.nnz_off[q + 1] - bt.nnz_off[q];
    });
    auto inst_lds = [&](int i) {
        return lds_bytes_for(bt.row_off[i + 1] - bt.row_off[i], bt.col_off[i + 1] - bt.col_off[i], sizeof(T));
    };
    int n_big = B, sm_m = 0, sm_n = 0;  // the wide launch's instance count; the narrow one's largest sizes
    if (o.batch_split > 0) {
        std::stable_partition(order.begin(), order.end(), [&](int i) { return inst_lds(i) > o.batch_split; });
        n_big = 0;
        for (int i : order)
            if (inst_lds(i) > o.batch_split) ++n_big;
        for (int k = n_big; k < B; ++k) {
            sm_m = std::max(sm_m, bt.row_off[order[k] + 1] - bt.row_off[order[k]]);
            sm_n = std::max(sm_n, bt.col_off[order[k] + 1] - bt.col_off[order[k]]);
        }
    }
    MIP_HIP(hipMemcpyAsync(w.hdr, hdr_running, sizeof(hdr_running), hipMemcpyHostToDevice, stream));
    MIP_HIP(hipMemcpyAsync(w.order, order.data(), B * 4, hipMemcpyHostToDevice, stream));
    MIP_HIP(hipMemcpyAsync(w.row_off, bt.row_off, (B + 1) * 4, hipMemcpyHostToDevice, stream));
    MIP_HIP(hipMemcpyAsync(w.eps, eps, (size_t)B * 8, hipMemcpyHostToDevice, stream));
    MIP_HIP(hipMemcpyAsync(w.col_off, bt.col_off, (B + 1) * 4, hipMemcpyHostToDevice, stream));
    if (o.validate && !o.resume &&
        (rc = validate_blockdiag(bt, rpa, rpat, w.tiles_a, w.tiles_at, w.row_off, w.col_off, w.flags, w.partials,
                                 w.red, stream)))
        return rc;
    BArgs<T, V> a;
    a.B = B;
    a.lds_m = max_m;
    a.lds_n = max_n;
    a.order = w.order;
    a.row_off = w.row_off;
    a.col_off = w.col_off;
    a.a_rowptr = lp.a_rowptr;
    a.a_col = lp.a_col;
    a.a_val = lp.a_val;
    a.at_rowptr = lp.at_rowptr;
    a.at_col = lp.at_col;
    a.at_val = lp.at_val;
    a.b = lp.b;
    a.c = lp.c;
    a.a_vs = (V*)w.a_vs;
    a.at_vs = (V*)w.at_vs;
    a.a_cl = w.a_cl;
    a.at_cl = w.at_cl;
    a.x = (T*)w.x;
    a.x0 = (T*)w.x0;
    a.xhat = (T*)w.xhat;
    a.ct = (T*)w.ct;
    a.y0 = (T*)w.y0;
    a.yhat = (T*)w.yhat;
    a.bt = (T*)w.bt;
    a.d_row = w.d_row;
    a.d_col = w.d_col;
    a.pu = w.pu;
    a.pav = w.pav;
    a.xo = x;
    a.yo = y;
    a.zo = z;
    a.rpo = r_p;
    a.rdo = r_d;
    a.info = w.info;
    a.state = w.state;
    a.ysave = (T*)w.ysave;
    a.resume = o.resume;
    a.block_iters = o.batch_block_iters;
    a.counter = w.counter;
    a.eps = w.eps;
    a.step_safety = o.step_safety;
    a.rho = o.reflect_rho;
    a.beta_suff = o.beta_suff;
    a.beta_nec = o.beta_nec;
    a.beta_art = o.beta_art;
    a.theta = o.pw_theta;
    a.max_iter = o.max_iter;
    a.ruiz = o.ruiz_iters;
    a.pc = o.pock_chambolle;
    a.power_iters = o.power_iters;
    a.eval_every = o.eval_every;
    a.halpern = o.halpern;
    a.restarts = o.restarts;
    // persistent grids: as many workgroups as fit, never more than instances
    int dev = 0, cus = 256;
    MIP_HIP(hipGetDevice(&dev));
    MIP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    auto* k_narrow = k_batched<T, V, Acc, kBatchBlock>;
    auto* k_wide = k_batched<T, V, Acc, kBatchWide>;
    MIP_HIP(hipFuncSetAttribute((const void*)k_narrow, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    MIP_HIP(hipFuncSetAttribute((const void*)k_wide, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    auto grid_for_lds = [&](bool wide, int bytes, int count, int* g) {
        int per_cu = 1;
        if (wide) MIP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_wide, kBatchWide, bytes));
        else MIP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_narrow, kBatchBlock, bytes));
        *g = std::max(1, std::min(count, cus * std::max(per_cu, 1)));
        return 0;
    };
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, stream, w.counter, 64);
    const auto t1 = clk::now();
    hipEvent_t e0, e1;
    MIP_HIP(hipEventCreate(&e0));
    MIP_HIP(hipEventCreate(&e1));
    MIP_HIP(hipEventRecord(e0, stream));
    if (o.batch_split == 0) {
        int grid = 1;
        if ((rc = grid_for_lds(false, lds, B, &grid))) return rc;
        hipLaunchKernelGGL((k_batched<T, V, Acc, kBatchBlock>), dim3(grid), dim3(kBatchBlock), lds, stream, a);
        MIP_LAUNCH_CHECK();
    } else {
        // the small instances on a side stream at their occupancy, the others
        // (if any) on the caller's stream in wide workgroups at the largest
        // instance's occupancy; both persistent launches run at once and share
        // the CUs
        struct Side {
            hipStream_t s = nullptr;
            hipEvent_t fork = nullptr, join = nullptr;
            ~Side() {
                if (fork) (void)hipEventDestroy(fork);
                if (join) (void)hipEventDestroy(join);
                if (s) (void)hipStreamDestroy(s);
            }
        } side;
        MIP_HIP(hipStreamCreateWithFlags(&side.s, hipStreamNonBlocking));
        MIP_HIP(hipEventCreateWithFlags(&side.fork, hipEventDisableTiming));
        MIP_HIP(hipEventCreateWithFlags(&side.join, hipEventDisableTiming));
        MIP_HIP(hipEventRecord(side.fork, stream));
        MIP_HIP(hipStreamWaitEvent(side.s, side.fork, 0));
        BArgs<T, V> as = a;
        as.B = B - n_big;
        as.order = w.order + n_big;
        as.counter = w.counter + 1;
        as.lds_m = sm_m;
        as.lds_n = sm_n;
        const int lds_sm = lds_bytes_for(sm_m, sm_n, sizeof(T));
        // grids sized to be resident together: at most one wide workgroup
        // per CU, the narrow launch in what that leaves of the CU's threads
        // and LDS (neither launch waits on the other, so this is for speed
        // only)
        int max_thr = 2048, cu_lds = 160 * 1024;
        MIP_HIP(hipDeviceGetAttribute(&max_thr, hipDeviceAttributeMaxThreadsPerMultiProcessor, dev));
        MIP_HIP(hipDeviceGetAttribute(&cu_lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev));
        const bool shared = n_big > 0 && as.B > 0;
        if (n_big > 0) {
            BArgs<T, V> ab = a;
            ab.B = n_big;
            int grid = 1;
            if ((rc = grid_for_lds(true, lds, n_big, &grid))) return rc;
            if (shared) grid = std::min(grid, cus);
            hipLaunchKernelGGL((k_batched<T, V, Acc, kBatchWide>), dim3(grid), dim3(kBatchWide), lds, stream, ab);
            MIP_LAUNCH_CHECK();
        }
        if (as.B > 0) {
            int grid = 1;
            if ((rc = grid_for_lds(false, lds_sm, as.B, &grid))) return rc;
            if (shared) {
                const int by_thr = (max_thr - kBatchWide) / kBatchBlock;
                const int by_lds = lds_sm > 0 ? (cu_lds - lds) / lds_sm : by_thr;
                const int per_cu = std::max(1, std::min(grid / std::max(cus, 1), std::min(by_thr, by_lds)));
                grid = std::max(1, std::min(as.B, cus * per_cu));
            }
            hipLaunchKernelGGL((k_batched<T, V, Acc, kBatchBlock>), dim3(grid), dim3(kBatchBlock), lds_sm, side.s,
                               as);
            MIP_LAUNCH_CHECK();
        }
        MIP_HIP(hipEventRecord(side.join, side.s));
        MIP_HIP(hipStreamWaitEvent(stream, side.join, 0));
        MIP_HIP(hipStreamSynchronize(side.s));
    }
    MIP_HIP(hipEventRecord(e1, stream));
    MIP_HIP(hipMemcpyAsync(w.hdr, hdr_done, sizeof(hdr_done), hipMemcpyHostToDevice, stream));
    std::vector<BInst> res(B);
    MIP_HIP(hipMemcpyAsync(res.data(), w.info, sizeof(BInst) * B, hipMemcpyDeviceToHost, stream));
    MIP_HIP(hipStreamSynchronize(stream));
    float kms = 0.f;
    MIP_HIP(hipEventElapsedTime(&kms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const auto t2 = clk::now();
    int worst = MIPDHG_OPTIMAL;
    for (int i = 0; i < B; ++i) worst = std::max(worst, res[i].status);
    if (info) {
        for (int i = 0; i < B; ++i) {
            const BInst& r = res[i];
            mipdhg_info& f = info[i];
            memset(&f, 0, sizeof(f));
            f.status = r.status;
            f.restarts = r.restarts;
            f.iters = r.iters;
            f.rp_norm = sqrt(r.rp2);
            f.rd_norm = sqrt(r.rd2);
            f.pobj = r.pobj;
            f.dobj = r.dobj;
            f.gap = fabs(r.pobj - r.dobj);
            f.b_norm = r.b_norm;
            f.c_norm = r.c_norm;
            f.rel_rp = f.rp_norm / (1.0 + r.b_norm);
            f.rel_rd = f.rd_norm / (1.0 + r.c_norm);
            f.rel_gap = f.gap / (1.0 + fabs(r.pobj) + fabs(r.dobj));
            f.rp_inf = r.rp_inf;
            f.rd_inf = r.rd_inf;
            f.xz = r.xz;
            f.max_violation = std::max(std::max(r.rp_inf, r.rd_inf), r.xz / (1.0 + fabs(r.pobj)));
            f.sigma_hat = r.sigma_hat;
            f.eta = r.eta;
            f.omega0 = r.omega0;
            f.omega = r.omega;
            f.ms_setup = std::chrono::duration<double, std::milli>(t1 - t0).count();
            f.ms_iter = kms;
            f.ms_total = std::chrono::duration<double, std::milli>(t2 - t0).count();
        }
    }
    return worst;
}

}  // namespace mip

using namespace mip;

extern "C" int mipdhg_batch_workspace_size(const mipdhg_batch* bt, const mipdhg_options* opt, size_t* bytes) {
    clear_error();
    if (!bytes || !opt) return set_error("NULL argument"), MIPDHG_ERR_INVALID_ARG;
    int rc = check_batch(bt);
    if (rc) return rc;
    if ((rc = check_options(opt))) return rc;
    *bytes = carve_batch(nullptr, 0, bt->count, bt->whole.m, bt->whole.n, bt->whole.nnz, opt->precision).bytes;
    return 0;
}

extern "C" int mipdhg_solve_batched(const mipdhg_batch* bt, const mipdhg_options* opt, const double* eps_rel,
                                    void* workspace, size_t workspace_bytes, void* stream, double* x, double* y,
                                    double* z, double* r_p, double* r_d, mipdhg_info* info) {
    clear_error();
    int rc = check_batch(bt);
    if (rc) return rc;
    if (!opt) return set_error("options are NULL"), MIPDHG_ERR_INVALID_ARG;
    if ((rc = check_options(opt))) return rc;
    if (!eps_rel) return set_error("eps_rel (one per instance) is NULL"), MIPDHG_ERR_INVALID_ARG;
    for (int i = 0; i < bt->count; ++i)
        if (!(eps_rel[i] >= 0.0) || !std::isfinite(eps_rel[i]))
            return set_error("eps_rel[%d] must be finite and >= 0", i), MIPDHG_ERR_INVALID_ARG;
    if (!workspace || !x || !y || !z || !r_p || !r_d)
        return set_error("workspace and all five outputs are required"), MIPDHG_ERR_INVALID_ARG;
    if (is_general(bt->whole))
        return set_error("the general form (bounds, inequality rows) is a single-LP option"), MIPDHG_ERR_UNSUPPORTED;
    if (opt->pw_ki != 0.0 || opt->pw_kd != 0.0 || opt->restart_avg || opt->step_rule)
        return set_error("the PID primal weight, restart to average and the adaptive step are single-LP options"),
               MIPDHG_ERR_UNSUPPORTED;
    if (opt->trace_iters || opt->x_init || opt->y_init || opt->kernel_timing)
        return set_error("tracing, warm starts and kernel timing are single-LP options"), MIPDHG_ERR_UNSUPPORTED;
    if (opt->precision == MIPDHG_FP32_A)
        return set_error("FP32_A is a single-LP precision mode"), MIPDHG_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    switch (opt->precision) {
        case MIPDHG_FP64:
            return batched_impl<double, double, double>(*bt, *opt, eps_rel, workspace, workspace_bytes, s, x, y, z,
                                                        r_p, r_d, info);
        case MIPDHG_FP32:
            return batched_impl<float, float, double>(*bt, *opt, eps_rel, workspace, workspace_bytes, s, x, y, z, r_p,
                                                      r_d, info);
        case MIPDHG_FP32_BF16A:
            return batched_impl<float, uint16_t, double>(*bt, *opt, eps_rel, workspace, workspace_bytes, s, x, y, z,
                                                         r_p, r_d, info);
        default:
            return batched_impl<float, float, float>(*bt, *opt, eps_rel, workspace, workspace_bytes, s, x, y, z, r_p,
                                                     r_d, info);
    }
}

extern "C" int mipdhg_autotune_batched(const mipdhg_batch* bt, mipdhg_options* opt, const double* eps_rel,
                                       void* workspace, size_t workspace_bytes, void* stream, double* x, double* y,
                                       double* z, double* r_p, double* r_d, double* best_ms) {
    clear_error();
    int rc = check_batch(bt);
    if (rc) return rc;
    if (!opt) return set_error("options are NULL"), MIPDHG_ERR_INVALID_ARG;
    std::vector<mipdhg_info> info((size_t)bt->count);
    // LDS budgets of the narrow launch (0: one launch); the default stays
    // unless another is more than 3 % faster, so that the choice is stable
    const int32_t cands[] = {0, 2048, 4096, 8192, 16384, 32768};
    double best = 1e300, def = 1e300;
    int32_t pick = 0;
    for (int32_t c : cands) {
        mipdhg_options o = *opt;
        o.batch_split = c;
        o.resume = 0;  // whole solves from the start
        o.batch_block_iters = 0;
        const int r = mipdhg_solve_batched(bt, &o, eps_rel, workspace, workspace_bytes, stream, x, y, z, r_p, r_d,
                                           info.data());
        if (r < 0) return r;
        const double ms = info[0].ms_iter;  // the launches, timed by events on the stream
        if (c == 0) def = ms;
        if (ms < best) {
            best = ms;
            pick = c;
        }
    }
    if (best * 1.03 >= def) {
        pick = 0;
        best = def;
    }
    opt->batch_split = pick;
    if (best_ms) *best_ms = best;
    return 0;
}
