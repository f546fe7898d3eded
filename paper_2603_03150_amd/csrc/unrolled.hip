// The differentiable unrolled map x_K(c, b) and its hand-written adjoint.
//
// Forward: exactly K PDHG iterations per instance from (0, 0), with the same
// scaling, step and restart rule as the solve but no termination test.  The
// restart iterations and the (tau, sigma) of every epoch are recorded on a
// tape, together with a checkpoint of the state (x, y, x0, y0, k, epoch)
// every `ckpt` iterations.  x_K is the projected primal point of iteration K,
// unscaled.  The schedule and the steps are constants of the map (they are not
// differentiated), so x_K is piecewise linear in (c, b).
//
// Backward: for each checkpoint segment, last to first, the segment is
// recomputed from its checkpoint (bitwise identical to the forward pass),
// keeping the projection masks 1[x - tau g > 0] as one bit per column
// (wavefront ballots) plus k, tau and sigma of every iteration; then the
// segment is swept backwards.  One reverse step is the transpose of the
// iteration's linearisation:
//   Halpern / restart:  adjoints of x_hat, y_hat from the adjoints of the new
//                       state and anchor (a restart sends both to x_hat, y_hat)
//   dual step:          lam_y += lam_yhat, lam_b~ += sigma lam_yhat,
//                       lam_xbar = -sigma A~^T lam_yhat
//   extrapolation:      lam_xhat += 2 lam_xbar, lam_x -= lam_xbar
//   projection:         lam_v = mask * lam_xhat
//   primal step:        lam_x += lam_v, lam_g = -tau lam_v, lam_c~ += lam_g,
//                       lam_y -= A~ lam_g
// with the seed D_c * grad(x_K) on the last x_hat.  dL/dc = D_c lam_c~ and
// dL/db = D_r lam_b~.  Both passes run one workgroup per instance in one
// persistent launch, with the two gathered vectors in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.h"
#include "inst_common.h"
#include "plain.h"

namespace mip {

template <typename T, typename V>
struct UArgs {
    int32_t B, K, ckpt, E, nseg, nep, W;
    int32_t lds_m, lds_n, replay;
    int32_t N, Mrows;
    const int32_t *row_off, *col_off, *word_off;
    InstMat M;
    // tape: scaling, scaled values, schedule, checkpoints
    double *d_row, *d_col, *pu, *pav;
    V *a_vs, *at_vs;
    uint16_t *a_cl, *at_cl;  // instance-local columns of A, A^T
    T *bt, *ct;
    double *eta, *omega0, *taus, *sigmas;
    int8_t* restart;
    T *cp_x, *cp_x0, *cp_y, *cp_y0;
    int32_t *cp_k, *cp_ep;
    // working state
    T *x, *x0, *y0, *xhat, *yhat;
    // backward
    uint64_t* masks;
    int32_t* kbuf;
    double *tbuf, *sbuf;
    T *lx, *lx0, *ly, *ly0;
    double *lct, *lbt;
    const double* gx;
    double *xK, *gc, *gb;
    int32_t* counter;
    double step_safety, rho, beta_suff, beta_nec, beta_art, theta;
    int32_t ruiz, pc, power_iters, halpern, restarts;
};

template <typename T, typename V>
struct UInst {
    int inst, r0, r1, c0, c1, m, n;
};

// One forward iteration t of instance u with step (tau, sig) and Halpern
// weight from k.  With masks != nullptr the projection masks are stored.
// Returns q = (||x-x^||^2, ||x^-x0||^2, ||y-y^||^2, ||y^-y0||^2) partials of
// this thread when `want_q`.
template <typename T, typename V, typename Acc>
__device__ __forceinline__ void u_iterate(const UArgs<T, V>& a, const UInst<T, V>& u, T* yL, T* xbL, int64_t k,
                                          double tau, double sig, bool want_q, bool keep_hat, bool last,
                                          uint64_t* maskrow, double (&q)[4]) {
    const int tid = threadIdx.x;
    const double w = a.halpern ? (double)(k + 1) / (double)(k + 2) : 1.0;
    const double omw = 1.0 - w, rho = a.rho, opr = 1.0 + a.rho;
    // the next row's bounds and vector entries are loaded (branch-free,
    // clamped to the last row) while this row is summed
    int nb0 = 0, nb1 = 0;
    T nx = 0, nx0 = 0, nct = 0;
    if (u.n > 0) {
        const int g = u.c0 + min(tid, u.n - 1);
        nb0 = a.M.at_rowptr[g];
        nb1 = a.M.at_rowptr[g + 1];
        nx = a.x[g];
        nx0 = a.x0[g];
        nct = a.ct[g];
    }
    for (int j = tid; j < u.n; j += kBatchBlock) {
        const int g = u.c0 + j;
        const int b0 = nb0, b1 = nb1;
        const double o = (double)nx, an = (double)nx0, ctg = (double)nct;
        {
            const int gn = u.c0 + min(j + kBatchBlock, u.n - 1);
            nb0 = a.M.at_rowptr[gn];
            nb1 = a.M.at_rowptr[gn + 1];
            nx = a.x[gn];
            nx0 = a.x0[gn];
            nct = a.ct[gn];
        }
        const Acc s = row_dot4<Acc>(a.at_vs, a.at_cl, yL, b0, b1);
        const double v = o - tau * (ctg - (double)s);
        const double hh = v < 0.0 ? 0.0 : v;
        if (maskrow) {
            const unsigned long long bits = __ballot(v > 0.0);
            if ((tid & (kWave - 1)) == 0) maskrow[j >> 6] = bits;
        }
        xbL[j] = (T)(2.0 * hh - o);
        a.x[g] = (T)(w * (opr * hh - rho * o) + omw * an);
        if (want_q) {
            const double d = o - hh, e = hh - an;
            q[0] += d * d;
            q[1] += e * e;
        }
        if (keep_hat) a.xhat[g] = (T)hh;
        if (last) a.xK[g] = a.d_col[g] * hh;
    }
    __syncthreads();
    int mb0 = 0, mb1 = 0;
    T my0 = 0, mbt = 0;
    if (u.m > 0) {
        const int g = u.r0 + min(tid, u.m - 1);
        mb0 = a.M.a_rowptr[g];
        mb1 = a.M.a_rowptr[g + 1];
        my0 = a.y0[g];
        mbt = a.bt[g];
    }
    for (int i = tid; i < u.m; i += kBatchBlock) {
        const int g = u.r0 + i;
        const int b0 = mb0, b1 = mb1;
        const double an = (double)my0, btg = (double)mbt;
        {
            const int gn = u.r0 + min(i + kBatchBlock, u.m - 1);
            mb0 = a.M.a_rowptr[gn];
            mb1 = a.M.a_rowptr[gn + 1];
            my0 = a.y0[gn];
            mbt = a.bt[gn];
        }
        const Acc s = row_dot4<Acc>(a.a_vs, a.a_cl, xbL, b0, b1);
        const double o = (double)yL[i];
        const double hh = o + sig * (btg - (double)s);
        yL[i] = (T)(w * (opr * hh - rho * o) + omw * an);
        if (want_q) {
            const double d = o - hh, e = hh - an;
            q[2] += d * d;
            q[3] += e * e;
        }
        if (keep_hat) a.yhat[g] = (T)hh;
    }
    __syncthreads();
}

// state and anchor <- projected point (a restart)
template <typename T, typename V>
__device__ __forceinline__ void u_restart(const UArgs<T, V>& a, const UInst<T, V>& u, T* yL) {
    for (int j = threadIdx.x; j < u.n; j += kBatchBlock) {
        const T v = a.xhat[u.c0 + j];
        a.x[u.c0 + j] = v;
        a.x0[u.c0 + j] = v;
    }
    for (int i = threadIdx.x; i < u.m; i += kBatchBlock) {
        const T v = a.yhat[u.r0 + i];
        yL[i] = v;
        a.y0[u.r0 + i] = v;
    }
    __syncthreads();
}

template <typename T, typename V, typename Acc>
__device__ void forward_instance(const UArgs<T, V>& a, const UInst<T, V>& u, T* yL, T* xbL, double* sh) {
    const int tid = threadIdx.x, i = u.inst, B = a.B;
    const InstSetup su = inst_setup<T, V>(a.M, u.r0, u.r1, u.c0, u.c1, a.d_row, a.d_col, a.pu, a.pav,
                                          a.a_vs, a.at_vs, a.a_cl, a.at_cl, a.bt, a.ct, a.ruiz, a.pc,
                                          a.power_iters, a.step_safety, xbL, yL, sh);
    double omega = su.omega0;
    int epoch = 0;
    double tau, sig;
    if (a.replay) {
        tau = a.taus[i];
        sig = a.sigmas[i];
    } else {
        tau = su.eta / omega;
        sig = su.eta * omega;
        if (tid == 0) {
            a.eta[i] = su.eta;
            a.omega0[i] = su.omega0;
            a.taus[i] = tau;
            a.sigmas[i] = sig;
        }
    }
    for (int j = tid; j < u.n; j += kBatchBlock) {
        a.x[u.c0 + j] = (T)0;
        a.x0[u.c0 + j] = (T)0;
    }
    for (int r = tid; r < u.m; r += kBatchBlock) {
        yL[r] = (T)0;
        a.y0[u.r0 + r] = (T)0;
    }
    __syncthreads();
    int64_t k = 0;
    double R0 = NAN, R_prev = INFINITY;
    double nomax[1] = {0.0};
    for (int t = 1; t <= a.K; ++t) {
        if ((t - 1) % a.ckpt == 0) {  // checkpoint of the state before iteration t
            const int seg = (t - 1) / a.ckpt;
            for (int j = tid; j < u.n; j += kBatchBlock) {
                a.cp_x[(int64_t)seg * a.N + u.c0 + j] = a.x[u.c0 + j];
                a.cp_x0[(int64_t)seg * a.N + u.c0 + j] = a.x0[u.c0 + j];
            }
            for (int r = tid; r < u.m; r += kBatchBlock) {
                a.cp_y[(int64_t)seg * a.Mrows + u.r0 + r] = yL[r];
                a.cp_y0[(int64_t)seg * a.Mrows + u.r0 + r] = a.y0[u.r0 + r];
            }
            if (tid == 0) {
                a.cp_k[seg * B + i] = (int32_t)k;
                a.cp_ep[seg * B + i] = epoch;
            }
        }
        const bool at_eval = (t % a.E == 0) && t < a.K;
        const bool first = k == 0;
        const bool need_q = !a.replay && (first || at_eval);
        double q[4] = {0.0, 0.0, 0.0, 0.0};
        u_iterate<T, V, Acc>(a, u, yL, xbL, k, tau, sig, need_q, at_eval, t == a.K, nullptr, q);
        if (need_q) wg_reduce<4, 0>(q, nomax, sh);
        if (!a.replay && first) R0 = sqrt(omega * q[0] + q[2] / omega);
        ++k;
        if (!at_eval) continue;
        bool restart;
        if (a.replay) {
            restart = a.restart[(int64_t)(t - 1) * B + i] != 0;
        } else {
            const double R = sqrt(omega * q[0] + q[2] / omega);
            restart = a.restarts && ((R <= a.beta_suff * R0) || (R <= a.beta_nec * R0 && R > R_prev) ||
                                     ((double)k >= a.beta_art * (double)t));
            if (restart) {
                const double dx = sqrt(q[1]), dy = sqrt(q[3]);
                if (dx > 1e-10 && dy > 1e-10)
                    omega = exp(a.theta * log(dy / dx) + (1.0 - a.theta) * log(omega));
                R_prev = INFINITY;
            } else {
                R_prev = R;
            }
        }
        if (restart) {
            ++epoch;
            if (a.replay) {
                tau = a.taus[(int64_t)epoch * B + i];
                sig = a.sigmas[(int64_t)epoch * B + i];
            } else {
                tau = su.eta / omega;
                sig = su.eta * omega;
                if (tid == 0) {
                    a.restart[(int64_t)(t - 1) * B + i] = 1;
                    a.taus[(int64_t)epoch * B + i] = tau;
                    a.sigmas[(int64_t)epoch * B + i] = sig;
                }
            }
            u_restart<T, V>(a, u, yL);
            k = 0;
        }
    }
}

template <typename T, typename V, typename Acc>
__device__ void backward_instance(const UArgs<T, V>& a, const UInst<T, V>& u, T* yL, T* xbL) {
    const int tid = threadIdx.x, i = u.inst, B = a.B;
    for (int j = tid; j < u.n; j += kBatchBlock) {
        const int g = u.c0 + j;
        a.lx[g] = (T)0;
        a.lx0[g] = (T)0;
        a.lct[g] = 0.0;
    }
    for (int r = tid; r < u.m; r += kBatchBlock) {
        const int g = u.r0 + r;
        a.ly[g] = (T)0;
        a.ly0[g] = (T)0;
        a.lbt[g] = 0.0;
    }
    const double rho = a.rho, opr = 1.0 + a.rho;
    double qd[4];
    for (int seg = a.nseg - 1; seg >= 0; --seg) {
        const int tb = seg * a.ckpt, te = min(a.K, tb + a.ckpt);
        // restore the checkpoint and recompute the segment, keeping masks
        for (int j = tid; j < u.n; j += kBatchBlock) {
            a.x[u.c0 + j] = a.cp_x[(int64_t)seg * a.N + u.c0 + j];
            a.x0[u.c0 + j] = a.cp_x0[(int64_t)seg * a.N + u.c0 + j];
        }
        for (int r = tid; r < u.m; r += kBatchBlock) {
            yL[r] = a.cp_y[(int64_t)seg * a.Mrows + u.r0 + r];
            a.y0[u.r0 + r] = a.cp_y0[(int64_t)seg * a.Mrows + u.r0 + r];
        }
        int64_t k = a.cp_k[seg * B + i];
        int epoch = a.cp_ep[seg * B + i];
        __syncthreads();
        for (int t = tb + 1; t <= te; ++t) {
            const int it = t - tb - 1;
            const double tau = a.taus[(int64_t)epoch * B + i], sig = a.sigmas[(int64_t)epoch * B + i];
            if (tid == 0) {
                a.kbuf[(int64_t)it * B + i] = (int32_t)k;
                a.tbuf[(int64_t)it * B + i] = tau;
                a.sbuf[(int64_t)it * B + i] = sig;
            }
            const bool rs = a.restart[(int64_t)(t - 1) * B + i] != 0;
            u_iterate<T, V, Acc>(a, u, yL, xbL, k, tau, sig, false, rs, false,
                            a.masks + (int64_t)it * a.W + a.word_off[i], qd);
            ++k;
            if (rs) {
                u_restart<T, V>(a, u, yL);
                k = 0;
                ++epoch;
            }
        }
        __syncthreads();  // kbuf / tbuf / sbuf written by thread 0 are read by all
        // reverse sweep over the segment; yL holds lam_yhat, xbL holds lam_g
        T* lyhL = yL;
        T* lgL = xbL;
        for (int t = te; t > tb; --t) {
            const int it = t - tb - 1;
            const bool rs = a.restart[(int64_t)(t - 1) * B + i] != 0;
            const int64_t kt = a.kbuf[(int64_t)it * B + i];
            const double w = a.halpern ? (double)(kt + 1) / (double)(kt + 2) : 1.0;
            const double omw = 1.0 - w;
            const double tau = a.tbuf[(int64_t)it * B + i], sig = a.sbuf[(int64_t)it * B + i];
            // (R1) rows: adjoint of y_hat, of the previous y (partial) and anchor
            for (int r = tid; r < u.m; r += kBatchBlock) {
                const int g = u.r0 + r;
                const double ly = (double)a.ly[g], ly0 = (double)a.ly0[g];
                const double lyh = rs ? ly + ly0 : w * opr * ly;
                lyhL[r] = (T)lyh;
                a.ly[g] = (T)((rs ? 0.0 : -w * rho * ly) + lyh);
                a.ly0[g] = (T)(rs ? 0.0 : ly0 + omw * ly);
                a.lbt[g] += sig * lyh;
            }
            __syncthreads();
            // (C) columns: lam_xbar = -sigma A~^T lam_yhat, then extrapolation,
            // projection and primal step
            const uint64_t* mrow = a.masks + (int64_t)it * a.W + a.word_off[i];
            for (int j = tid; j < u.n; j += kBatchBlock) {
                const int g = u.c0 + j;
                const Acc s =
                    row_dot4<Acc>(a.at_vs, a.at_cl, lyhL, a.M.at_rowptr[g], a.M.at_rowptr[g + 1]);
                const double lxbar = -sig * (double)s;
                const double lx = (double)a.lx[g], lx0 = (double)a.lx0[g];
                double lxh = (rs ? lx + lx0 : w * opr * lx) + 2.0 * lxbar;
                if (t == a.K) lxh += a.d_col[g] * a.gx[g];
                const bool on = (mrow[j >> 6] >> (j & 63)) & 1ull;
                const double lv = on ? lxh : 0.0;
                const double lg = -tau * lv;
                a.lx[g] = (T)((rs ? 0.0 : -w * rho * lx) - lxbar + lv);
                a.lx0[g] = (T)(rs ? 0.0 : lx0 + omw * lx);
                a.lct[g] += lg;
                lgL[j] = (T)lg;
            }
            __syncthreads();
            // (R2) rows: lam_y -= A~ lam_g
            for (int r = tid; r < u.m; r += kBatchBlock) {
                const int g = u.r0 + r;
                const Acc s = row_dot4<Acc>(a.a_vs, a.a_cl, lgL, a.M.a_rowptr[g], a.M.a_rowptr[g + 1]);
                a.ly[g] = (T)((double)a.ly[g] - (double)s);
            }
            __syncthreads();
        }
    }
    for (int j = tid; j < u.n; j += kBatchBlock) a.gc[u.c0 + j] = a.d_col[u.c0 + j] * a.lct[u.c0 + j];
    for (int r = tid; r < u.m; r += kBatchBlock) a.gb[u.r0 + r] = a.d_row[u.r0 + r] * a.lbt[u.r0 + r];
    __syncthreads();
}

template <typename T, typename V, typename Acc, bool BACKWARD>
__global__ __launch_bounds__(kBatchBlock) void k_unrolled(UArgs<T, V> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    T* yL = (T*)smem;
    T* xbL = yL + a.lds_m;
    __shared__ double sh[8 * (kBatchBlock / kWave)];
    __shared__ int next;
    while (true) {
        if (threadIdx.x == 0) next = atomicAdd(a.counter, 1);
        __syncthreads();
        const int qi = next;
        __syncthreads();
        if (qi >= a.B) break;
        UInst<T, V> u;
        u.inst = qi;
        u.r0 = a.row_off[qi];
        u.r1 = a.row_off[qi + 1];
        u.c0 = a.col_off[qi];
        u.c1 = a.col_off[qi + 1];
        u.m = u.r1 - u.r0;
        u.n = u.c1 - u.c0;
        if (BACKWARD) backward_instance<T, V, Acc>(a, u, yL, xbL);
        else forward_instance<T, V, Acc>(a, u, yL, xbL, sh);
    }
}

__global__ void k_zero_bytes(uint8_t* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct TapeLayout {
    int32_t *row_off, *col_off, *word_off, *counter;
    double *d_row, *d_col, *pu, *pav, *eta, *omega0, *taus, *sigmas;
    void *a_vs, *at_vs, *bt, *ct;
    uint16_t *a_cl, *at_cl;
    int8_t* restart;
    void *cp_x, *cp_x0, *cp_y, *cp_y0;
    int32_t *cp_k, *cp_ep;
    void *x, *x0, *y0, *xhat, *yhat;
    uint64_t* masks;
    int32_t* kbuf;
    double *tbuf, *sbuf;
    void *lx, *lx0, *ly, *ly0;
    double *lct, *lbt;
    int32_t *vtiles_a, *vtiles_at, *vflags;  // input validation (forward)
    double *vpartials, *vred;
    int32_t W, nseg, nep;
    size_t bytes;
};

static TapeLayout carve_tape(void* base, size_t cap, const mipdhg_batch& bt, int prec, int K, int ckpt, int E) {
    Carver cv(base, cap);
    TapeLayout t;
    const int64_t B = bt.count, m = bt.whole.m, n = bt.whole.n, nnz = bt.whole.nnz;
    const size_t vs = prec == MIPDHG_FP64 ? 8 : (prec == MIPDHG_FP32_BF16A ? 2 : 4);
    const size_t ts = prec == MIPDHG_FP64 ? 8 : 4;
    int64_t W = 0;
    for (int64_t i = 0; i < B; ++i) W += (bt.col_off[i + 1] - bt.col_off[i] + 63) / 64;
    t.W = (int32_t)W;
    t.nseg = (K + ckpt - 1) / ckpt;
    t.nep = (K - 1) / E + 2;
    t.row_off = cv.take<int32_t>(B + 1);
    t.col_off = cv.take<int32_t>(B + 1);
    t.word_off = cv.take<int32_t>(B + 1);
    t.counter = cv.take<int32_t>(64);
    t.d_row = cv.take<double>(m);
    t.d_col = cv.take<double>(n);
    t.pu = cv.take<double>(n);
    t.pav = cv.take<double>(m);
    t.eta = cv.take<double>(B);
    t.omega0 = cv.take<double>(B);
    t.taus = cv.take<double>((size_t)t.nep * B);
    t.sigmas = cv.take<double>((size_t)t.nep * B);
    t.a_vs = cv.take<char>(nnz * vs);
    t.at_vs = cv.take<char>(nnz * vs);
    t.a_cl = cv.take<uint16_t>(nnz);
    t.at_cl = cv.take<uint16_t>(nnz);
    t.bt = cv.take<char>(m * ts);
    t.ct = cv.take<char>(n * ts);
    t.restart = cv.take<int8_t>((size_t)K * B);
    t.cp_x = cv.take<char>((size_t)t.nseg * n * ts);
    t.cp_x0 = cv.take<char>((size_t)t.nseg * n * ts);
    t.cp_y = cv.take<char>((size_t)t.nseg * m * ts);
    t.cp_y0 = cv.take<char>((size_t)t.nseg * m * ts);
    t.cp_k = cv.take<int32_t>((size_t)t.nseg * B);
    t.cp_ep = cv.take<int32_t>((size_t)t.nseg * B);
    t.x = cv.take<char>(n * ts);
    t.x0 = cv.take<char>(n * ts);
    t.y0 = cv.take<char>(m * ts);
    t.xhat = cv.take<char>(n * ts);
    t.yhat = cv.take<char>(m * ts);
    t.masks = cv.take<uint64_t>((size_t)ckpt * W);
    t.kbuf = cv.take<int32_t>((size_t)ckpt * B);
    t.tbuf = cv.take<double>((size_t)ckpt * B);
    t.sbuf = cv.take<double>((size_t)ckpt * B);
    t.lx = cv.take<char>(n * ts);
    t.lx0 = cv.take<char>(n * ts);
    t.ly = cv.take<char>(m * ts);
    t.ly0 = cv.take<char>(m * ts);
    t.lct = cv.take<double>(n);
    t.lbt = cv.take<double>(m);
    const int64_t vs_slots = blockdiag_tile_slots(m, n, nnz);
    t.vtiles_a = cv.take<int32_t>(4 * vs_slots);
    t.vtiles_at = cv.take<int32_t>(4 * vs_slots);
    t.vflags = cv.take<int32_t>(64);
    t.vpartials = cv.take<double>((size_t)vs_slots + 16);
    t.vred = cv.take<double>(16);
    t.bytes = (cv.off + 255) & ~size_t(255);
    return t;
}

static int check_unrolled(const mipdhg_batch* bt, const mipdhg_options* o, int K, int ckpt) {
    if (!bt || !o) return set_error("NULL argument"), MIPDHG_ERR_INVALID_ARG;
    if (bt->count < 1 || !bt->row_off || !bt->col_off || !bt->nnz_off)
        return set_error("batch count >= 1 and host offsets are required"), MIPDHG_ERR_INVALID_ARG;
    int rc = check_lp(&bt->whole);
    if (rc) return rc;
    if ((rc = check_options(o))) return rc;
    if (K < 1 || ckpt < 1) return set_error("K >= 1 and ckpt_every >= 1 required"), MIPDHG_ERR_INVALID_ARG;
    if (o->resume) return set_error("the unrolled map has no state to resume"), MIPDHG_ERR_UNSUPPORTED;
    if (is_general(bt->whole))
        return set_error("the general form (bounds, inequality rows) is a single-LP option"), MIPDHG_ERR_UNSUPPORTED;
    if (o->pw_ki != 0.0 || o->pw_kd != 0.0 || o->restart_avg || o->step_rule)
        return set_error("the PID primal weight, restart to average and the adaptive step are single-LP options"),
               MIPDHG_ERR_UNSUPPORTED;
    const int B = bt->count;
    if (bt->row_off[0] != 0 || bt->col_off[0] != 0 || bt->nnz_off[0] != 0 || bt->row_off[B] != bt->whole.m ||
        bt->col_off[B] != bt->whole.n || bt->nnz_off[B] != bt->whole.nnz)
        return set_error("instance offsets must start at 0 and end at m, n, nnz"), MIPDHG_ERR_INVALID_ARG;
    for (int i = 0; i < B; ++i)
        if (bt->row_off[i + 1] <= bt->row_off[i] || bt->col_off[i + 1] <= bt->col_off[i])
            return set_error("instance %d is empty", i), MIPDHG_ERR_INVALID_ARG;
    return 0;
}

template <typename T, typename V, typename Acc>
static int unrolled_impl(const mipdhg_batch& bt, const mipdhg_options& o, int K, int ckpt, void* tape,
                         size_t tape_bytes, hipStream_t stream, bool backward, int replay, const double* gx,
                         double* out1, double* out2) {
    TapeLayout t = carve_tape(tape, tape_bytes, bt, o.precision, K, ckpt, o.eval_every);
    if (t.bytes > tape_bytes)
        return set_error("tape too small: %zu bytes given, %zu needed", tape_bytes, t.bytes), MIPDHG_ERR_WORKSPACE;
    if (((uintptr_t)tape & 255) != 0) return set_error("tape must be 256-byte aligned"), MIPDHG_ERR_INVALID_ARG;
    const int B = bt.count;
    int max_m = 0, max_n = 0;
    for (int i = 0; i < B; ++i) {
        max_m = std::max(max_m, bt.row_off[i + 1] - bt.row_off[i]);
        max_n = std::max(max_n, bt.col_off[i + 1] - bt.col_off[i]);
    }
    const int lds = (int)(((size_t)max_m + (size_t)max_n) * sizeof(T) + 16);
    if (lds > 150 * 1024 || max_m > kInstMaxDim || max_n > kInstMaxDim)
        return set_error("instance too large for LDS (%d bytes)", lds), MIPDHG_ERR_UNSUPPORTED;
    const mipdhg_lp& lp = bt.whole;
    if (!backward) {
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
        std::vector<int32_t> wo(B + 1, 0);
        for (int i = 0; i < B; ++i) wo[i + 1] = wo[i] + (bt.col_off[i + 1] - bt.col_off[i] + 63) / 64;
        MIP_HIP(hipMemcpyAsync(t.row_off, bt.row_off, (B + 1) * 4, hipMemcpyHostToDevice, stream));
        MIP_HIP(hipMemcpyAsync(t.col_off, bt.col_off, (B + 1) * 4, hipMemcpyHostToDevice, stream));
        MIP_HIP(hipMemcpyAsync(t.word_off, wo.data(), (B + 1) * 4, hipMemcpyHostToDevice, stream));
        // column ranges, finiteness, A^T against A, and the block-diagonal
        // structure, before any kernel indexes with the columns
        if (o.validate && (rc = validate_blockdiag(bt, rpa, rpat, t.vtiles_a, t.vtiles_at, t.row_off, t.col_off,
                                                   t.vflags, t.vpartials, t.vred, stream)))
            return rc;
        if (!replay)
            hipLaunchKernelGGL(k_zero_bytes, dim3(grid_for((int64_t)K * B)), dim3(kBlock), 0, stream,
                               (uint8_t*)t.restart, (int64_t)K * B);
        MIP_HIP(hipStreamSynchronize(stream));  // host vectors go out of scope
    }
    UArgs<T, V> a;
    memset(&a, 0, sizeof(a));
    a.B = B;
    a.K = K;
    a.ckpt = ckpt;
    a.E = o.eval_every;
    a.nseg = t.nseg;
    a.nep = t.nep;
    a.W = t.W;
    a.lds_m = max_m;
    a.lds_n = max_n;
    a.replay = replay;
    a.N = lp.n;
    a.Mrows = lp.m;
    a.row_off = t.row_off;
    a.col_off = t.col_off;
    a.word_off = t.word_off;
    a.M = InstMat{lp.a_rowptr, lp.a_col, lp.a_val, lp.at_rowptr, lp.at_col, lp.at_val, lp.b, lp.c};
    a.d_row = t.d_row;
    a.d_col = t.d_col;
    a.pu = t.pu;
    a.pav = t.pav;
    a.a_vs = (V*)t.a_vs;
    a.at_vs = (V*)t.at_vs;
    a.a_cl = t.a_cl;
    a.at_cl = t.at_cl;
    a.bt = (T*)t.bt;
    a.ct = (T*)t.ct;
    a.eta = t.eta;
    a.omega0 = t.omega0;
    a.taus = t.taus;
    a.sigmas = t.sigmas;
    a.restart = t.restart;
    a.cp_x = (T*)t.cp_x;
    a.cp_x0 = (T*)t.cp_x0;
    a.cp_y = (T*)t.cp_y;
    a.cp_y0 = (T*)t.cp_y0;
    a.cp_k = t.cp_k;
    a.cp_ep = t.cp_ep;
    a.x = (T*)t.x;
    a.x0 = (T*)t.x0;
    a.y0 = (T*)t.y0;
    a.xhat = (T*)t.xhat;
    a.yhat = (T*)t.yhat;
    a.masks = t.masks;
    a.kbuf = t.kbuf;
    a.tbuf = t.tbuf;
    a.sbuf = t.sbuf;
    a.lx = (T*)t.lx;
    a.lx0 = (T*)t.lx0;
    a.ly = (T*)t.ly;
    a.ly0 = (T*)t.ly0;
    a.lct = t.lct;
    a.lbt = t.lbt;
    a.gx = gx;
    a.xK = backward ? nullptr : out1;
    a.gc = backward ? out1 : nullptr;
    a.gb = backward ? out2 : nullptr;
    a.counter = t.counter;
    a.step_safety = o.step_safety;
    a.rho = o.reflect_rho;
    a.beta_suff = o.beta_suff;
    a.beta_nec = o.beta_nec;
    a.beta_art = o.beta_art;
    a.theta = o.pw_theta;
    a.ruiz = o.ruiz_iters;
    a.pc = o.pock_chambolle;
    a.power_iters = o.power_iters;
    a.halpern = o.halpern;
    a.restarts = o.restarts;
    int dev = 0, cus = 256, per_cu = 1;
    MIP_HIP(hipGetDevice(&dev));
    MIP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (backward) {
        MIP_HIP(hipFuncSetAttribute((const void*)k_unrolled<T, V, Acc, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    lds));
        MIP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_unrolled<T, V, Acc, true>, kBatchBlock, lds));
    } else {
        MIP_HIP(hipFuncSetAttribute((const void*)k_unrolled<T, V, Acc, false>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, lds));
        MIP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_unrolled<T, V, Acc, false>, kBatchBlock, lds));
    }
    const int grid = std::max(1, std::min(B, cus * std::max(per_cu, 1)));
    hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(64), 0, stream, (uint8_t*)t.counter, (int64_t)256);
    if (backward)
        hipLaunchKernelGGL((k_unrolled<T, V, Acc, true>), dim3(grid), dim3(kBatchBlock), lds, stream, a);
    else
        hipLaunchKernelGGL((k_unrolled<T, V, Acc, false>), dim3(grid), dim3(kBatchBlock), lds, stream, a);
    MIP_LAUNCH_CHECK();
    MIP_HIP(hipStreamSynchronize(stream));
    return 0;
}

}  // namespace mip

using namespace mip;

extern "C" int mipdhg_unrolled_tape_size(const mipdhg_batch* bt, const mipdhg_options* opt, int32_t K,
                                         int32_t ckpt_every, size_t* bytes) {
    clear_error();
    int rc = check_unrolled(bt, opt, K, ckpt_every);
    if (rc) return rc;
    if (!bytes) return set_error("bytes is NULL"), MIPDHG_ERR_INVALID_ARG;
    *bytes = carve_tape(nullptr, 0, *bt, opt->precision, K, ckpt_every, opt->eval_every).bytes;
    return 0;
}

extern "C" int mipdhg_unrolled_forward(const mipdhg_batch* bt, const mipdhg_options* opt, int32_t K,
                                       int32_t ckpt_every, int32_t replay, void* tape, size_t tape_bytes,
                                       void* stream, double* x_K) {
    clear_error();
    int rc = check_unrolled(bt, opt, K, ckpt_every);
    if (rc) return rc;
    if (!tape || !x_K) return set_error("tape and x_K are required"), MIPDHG_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (opt->precision == MIPDHG_FP32_A)
        return set_error("FP32_A is a single-LP precision mode"), MIPDHG_ERR_UNSUPPORTED;
    switch (opt->precision) {
        case MIPDHG_FP64:
            return unrolled_impl<double, double, double>(*bt, *opt, K, ckpt_every, tape, tape_bytes, s, false, replay,
                                                         nullptr, x_K, nullptr);
        case MIPDHG_FP32:
            return unrolled_impl<float, float, double>(*bt, *opt, K, ckpt_every, tape, tape_bytes, s, false, replay,
                                                       nullptr, x_K, nullptr);
        case MIPDHG_FP32_BF16A:
            return unrolled_impl<float, uint16_t, double>(*bt, *opt, K, ckpt_every, tape, tape_bytes, s, false,
                                                          replay, nullptr, x_K, nullptr);
        default:
            return unrolled_impl<float, float, float>(*bt, *opt, K, ckpt_every, tape, tape_bytes, s, false, replay,
                                                      nullptr, x_K, nullptr);
    }
}

extern "C" int mipdhg_unrolled_backward(const mipdhg_batch* bt, const mipdhg_options* opt, int32_t K,
                                        int32_t ckpt_every, void* tape, size_t tape_bytes, const double* grad_xK,
                                        void* stream, double* grad_c, double* grad_b) {
    clear_error();
    int rc = check_unrolled(bt, opt, K, ckpt_every);
    if (rc) return rc;
    if (!tape || !grad_xK || !grad_c || !grad_b)
        return set_error("tape, grad_xK, grad_c and grad_b are required"), MIPDHG_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (opt->precision == MIPDHG_FP32_A)
        return set_error("FP32_A is a single-LP precision mode"), MIPDHG_ERR_UNSUPPORTED;
    switch (opt->precision) {
        case MIPDHG_FP64:
            return unrolled_impl<double, double, double>(*bt, *opt, K, ckpt_every, tape, tape_bytes, s, true, 1,
                                                         grad_xK, grad_c, grad_b);
        case MIPDHG_FP32:
            return unrolled_impl<float, float, double>(*bt, *opt, K, ckpt_every, tape, tape_bytes, s, true, 1, grad_xK,
                                                       grad_c, grad_b);
        case MIPDHG_FP32_BF16A:
            return unrolled_impl<float, uint16_t, double>(*bt, *opt, K, ckpt_every, tape, tape_bytes, s, true, 1,
                                                          grad_xK, grad_c, grad_b);
        default:
            return unrolled_impl<float, float, float>(*bt, *opt, K, ckpt_every, tape, tape_bytes, s, true, 1, grad_xK,
                                                      grad_c, grad_b);
    }
}

extern "C" int mipdhg_unrolled_schedule(const mipdhg_batch* bt, const mipdhg_options* opt, int32_t K,
                                        int32_t ckpt_every, const void* tape, size_t tape_bytes, int32_t inst,
                                        void* stream, int32_t capacity, int32_t* restart_at, double* taus,
                                        double* sigmas, int32_t* n_restarts) {
    clear_error();
    int rc = check_unrolled(bt, opt, K, ckpt_every);
    if (rc) return rc;
    if (!tape || !restart_at || !taus || !sigmas || !n_restarts)
        return set_error("tape and the four outputs are required"), MIPDHG_ERR_INVALID_ARG;
    if (inst < 0 || inst >= bt->count) return set_error("inst must be in [0, count)"), MIPDHG_ERR_INVALID_ARG;
    const TapeLayout t = carve_tape(const_cast<void*>(tape), tape_bytes, *bt, opt->precision, K, ckpt_every,
                                    opt->eval_every);
    if (t.bytes > tape_bytes)
        return set_error("tape too small: %zu bytes given, %zu needed", tape_bytes, t.bytes), MIPDHG_ERR_WORKSPACE;
    const int B = bt->count;
    hipStream_t s = (hipStream_t)stream;
    std::vector<int8_t> flags((size_t)K * B);
    std::vector<double> tv((size_t)t.nep * B), sv((size_t)t.nep * B);
    MIP_HIP(hipMemcpyAsync(flags.data(), t.restart, flags.size(), hipMemcpyDeviceToHost, s));
    MIP_HIP(hipMemcpyAsync(tv.data(), t.taus, tv.size() * 8, hipMemcpyDeviceToHost, s));
    MIP_HIP(hipMemcpyAsync(sv.data(), t.sigmas, sv.size() * 8, hipMemcpyDeviceToHost, s));
    MIP_HIP(hipStreamSynchronize(s));
    int32_t nr = 0;
    for (int32_t it = 1; it <= K; ++it)
        if (flags[(size_t)(it - 1) * B + inst]) {
            if (nr + 1 >= capacity)
                return set_error("capacity %d holds fewer epochs than the schedule's", capacity),
                       MIPDHG_ERR_INVALID_ARG;
            restart_at[nr++] = it;
        }
    if (nr + 1 > capacity || nr + 1 > t.nep)
        return set_error("capacity %d holds fewer epochs than the schedule's", capacity), MIPDHG_ERR_INVALID_ARG;
    for (int32_t e = 0; e <= nr; ++e) {
        taus[e] = tv[(size_t)e * B + inst];
        sigmas[e] = sv[(size_t)e * B + inst];
    }
    *n_restarts = nr;
    return 0;
}
