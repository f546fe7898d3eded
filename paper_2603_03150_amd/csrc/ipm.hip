// Interior-point consumer of the centered start (Section 3.1): the solver
// Algorithm 1 hands its point to, and the alpha_min recovery loop around it.
//
// Mehrotra's primal-dual predictor-corrector (Wright 1997, Chapter 10) on the
// scaled LP min c~^T x s.t. A~ x = b~, x >= 0 with A~ = D_r A D_c, b~ = D_r b,
// c~ = D_c c.  Every Newton system goes through the normal equations
// (A~ D A~^T) dy = r_b - A~ (Z^-1 r_xz - D r_c), D = X Z^-1: the m x m matrix
// is formed dense on the device (each entry a merge of two sorted rows of A~,
// one thread per entry, fixed order), factored by a blocked right-looking
// Cholesky (64 x 64 blocks: a one-workgroup diagonal factor, a row-per-thread
// panel solve, an LDS-tiled trailing update), and the two triangular solves
// run in one workgroup, one wave doing each diagonal block with shuffles.
// The predictor and the corrector share the factor.  Scalars (norms, step
// lengths, mu) are fixed-order reductions read back by the host, which runs
// the iteration.  Dense factors bound m (kIpmMaxM): this consumer is for the
// modest LPs on which the paper's iteration-count ratio is measured, not for
// the large sparse models of Section 4, which need a sparse factorization.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "mipdhg.h"
#include "plain.h"

namespace mip {
namespace {

constexpr int kNb = 64;           // Cholesky block
constexpr int kIpmMaxM = 16384;   // dense normal matrix: 2 GiB at this size
constexpr int kRedBlocks = 1024;  // partial slots of a reduction

// out[r] = (s0 ? s0[r] : 0) + sgn * sum_k a_rk v[col_k] - (s1 ? s1[r] : 0);
// one wave per row, the lanes' strided sums added by a butterfly
__global__ __launch_bounds__(kBlock) void k_ipm_spmv(const int32_t* rp, const int32_t* col, const double* val,
                                                     const double* v, int32_t nrows, const double* s0, double sgn,
                                                     const double* s1, double* out) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t r = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (r >= nrows) return;
    double acc = 0.0;
    for (int k = rp[r] + lane; k < rp[r + 1]; k += kWave) acc += val[k] * v[col[k]];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
    if (lane == 0) out[r] = (s0 ? s0[r] : 0.0) + sgn * acc - (s1 ? s1[r] : 0.0);
}

// scaled values (d_row[i] a_ij) d_col[j]; trans: the rows are A's columns
__global__ void k_ipm_scale_vals(const int32_t* rp, const int32_t* col, const double* val, int32_t nrows,
                                 const double* d_row, const double* d_col, int trans, double* out) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * blockDim.x)
        for (int k = rp[r]; k < rp[r + 1]; ++k) {
            const int32_t c = col[k];
            const double dr = d_row ? d_row[trans ? c : r] : 1.0, dc = d_col ? d_col[trans ? r : c] : 1.0;
            out[k] = (dr * val[k]) * dc;
        }
}

// out = d .* v (either may be NULL for ones), or v / d (div)
__global__ void k_ipm_vscale(const double* v, const double* d, int div, int64_t n, double* out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double s = d ? d[i] : 1.0;
        out[i] = div ? v[i] / s : v[i] * s;
    }
}

// Lower triangle of M = A~ diag(w) A~^T (w NULL: ones): entry (i, k), k <= i,
// by merging the sorted columns of rows i and k.
__global__ __launch_bounds__(kBlock) void k_ipm_normal(const int32_t* rp, const int32_t* col, const double* val,
                                                       const double* w, int32_t m, double* M) {
    const int32_t i = blockIdx.y;
    const int32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k > i) return;
    int p = rp[i], q = rp[k];
    const int pe = rp[i + 1], qe = rp[k + 1];
    double s = 0.0;
    while (p < pe && q < qe) {
        const int32_t a = col[p], b = col[q];
        if (a == b) {
            s += (val[p] * (w ? w[a] : 1.0)) * val[q];
            ++p;
            ++q;
        } else if (a < b) {
            ++p;
        } else {
            ++q;
        }
    }
    M[(int64_t)i * m + k] = s;
}

// --- blocked Cholesky, lower triangle of a row-major m x m matrix in place.
// A pivot that is not positive (or underflows) is replaced by 1e128, which
// decouples that row (the usual treatment of a rank-deficient normal matrix);
// such replacements are counted in *flag.

// the nb x nb diagonal block at (k0, k0), one workgroup
__global__ __launch_bounds__(kBlock) void k_chol_diag(double* M, int32_t m, int32_t k0, int32_t nb, int32_t* flag) {
    __shared__ double L[kNb][kNb + 1];
    for (int e = threadIdx.x; e < kNb * kNb; e += kBlock) {
        const int i = e / kNb, j = e % kNb;
        L[i][j] = (i < nb && j <= i) ? M[(int64_t)(k0 + i) * m + k0 + j] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        if (threadIdx.x == 0) {
            double d = L[j][j];
            if (!(d > 1e-300)) {
                d = 1e128;
                atomicAdd(flag, 1);
            }
            L[j][j] = sqrt(d);
        }
        __syncthreads();
        for (int i = j + 1 + threadIdx.x; i < nb; i += kBlock) L[i][j] /= L[j][j];
        __syncthreads();
        // trailing part of the block: L[i][c] -= L[i][j] L[c][j], j < c <= i < nb
        const int w = nb - j - 1;
        for (int e = threadIdx.x; e < w * w; e += kBlock) {
            const int i = j + 1 + e / w, c = j + 1 + e % w;
            if (c <= i) L[i][c] -= L[i][j] * L[c][j];
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < kNb * kNb; e += kBlock) {
        const int i = e / kNb, j = e % kNb;
        if (i < nb && j <= i) M[(int64_t)(k0 + i) * m + k0 + j] = L[i][j];
    }
}

// rows below the block: X L11^T = A21, one row per thread (forward substitution)
__global__ __launch_bounds__(kBlock) void k_chol_panel(double* M, int32_t m, int32_t k0, int32_t nb) {
    __shared__ double L[kNb][kNb + 1];
    for (int e = threadIdx.x; e < kNb * kNb; e += kBlock) {
        const int i = e / kNb, j = e % kNb;
        L[i][j] = (i < nb && j <= i) ? M[(int64_t)(k0 + i) * m + k0 + j] : 0.0;
    }
    __syncthreads();
    const int64_t i = (int64_t)k0 + nb + (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    double* row = M + i * m + k0;
    double x[kNb];
#pragma unroll
    for (int j = 0; j < kNb; ++j) x[j] = j < nb ? row[j] : 0.0;
#pragma unroll
    for (int j = 0; j < kNb; ++j) {
        if (j < nb) {
            double s = x[j];
            for (int l = 0; l < j; ++l) s -= x[l] * L[j][l];
            x[j] = s / L[j][j];
        }
    }
#pragma unroll
    for (int j = 0; j < kNb; ++j)
        if (j < nb) row[j] = x[j];
}

// trailing update M[i][j] -= sum_l L[i][k0 + l] L[j][k0 + l] over the lower
// tiles (bi >= bj) of the region from k1 = k0 + nb; 64 x 64 tile per
// workgroup, 4 x 4 outputs per thread
__global__ __launch_bounds__(kBlock) void k_chol_update(double* M, int32_t m, int32_t k0, int32_t nb) {
    constexpr int kL = kNb / 2;  // columns of the panel staged at a time (two 16 KB halves)
    __shared__ double Pi[kL][kNb];  // Pi[l][a] = L[r0 + a][k0 + lc + l]
    __shared__ double Pj[kL][kNb];
    // linear tile index -> (bi, bj), bj <= bi
    const int64_t t = blockIdx.x;
    int64_t bi = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    while (bi * (bi + 1) / 2 > t) --bi;
    const int64_t bj = t - bi * (bi + 1) / 2;
    const int64_t k1 = (int64_t)k0 + nb;
    const int64_t r0 = k1 + bi * kNb, c0 = k1 + bj * kNb;
    const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;  // rows ty + 16 u, cols tx + 16 v
    double acc[4][4] = {};
    for (int lc = 0; lc < nb; lc += kL) {
        for (int e = threadIdx.x; e < kNb * kL; e += kBlock) {
            const int a = e / kL, l = e % kL;
            const bool in = lc + l < nb;
            Pi[l][a] = (r0 + a < m && in) ? M[(r0 + a) * m + k0 + lc + l] : 0.0;
            Pj[l][a] = (c0 + a < m && in) ? M[(c0 + a) * m + k0 + lc + l] : 0.0;
        }
        __syncthreads();
        for (int l = 0; l < kL; ++l) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = Pi[l][ty + 16 * u];
#pragma unroll
            for (int v = 0; v < 4; ++v) b[v] = Pj[l][tx + 16 * v];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t i = r0 + ty + 16 * u, j = c0 + tx + 16 * v;
            if (i < m && j <= i) M[i * m + j] -= acc[u][v];
        }
}

// L x = b in place (x holds b), one workgroup
__global__ __launch_bounds__(kBlock) void k_trsv_lower(const double* L, int32_t m, double* x) {
    const int lane = threadIdx.x;
    for (int32_t k0 = 0; k0 < m; k0 += kNb) {
        const int nb = min(kNb, m - k0);
        if (threadIdx.x < kWave) {
            double xi = lane < nb ? x[k0 + lane] : 0.0, mine = 0.0;
            for (int j = 0; j < nb; ++j) {
                const double xj = __shfl(xi, j, kWave) / L[(int64_t)(k0 + j) * m + k0 + j];
                if (lane == j) mine = xj;
                if (lane > j && lane < nb) xi -= L[(int64_t)(k0 + lane) * m + k0 + j] * xj;
            }
            if (lane < nb) x[k0 + lane] = mine;
        }
        __syncthreads();
        for (int64_t i = (int64_t)k0 + nb + threadIdx.x; i < m; i += kBlock) {
            const double* row = L + i * m + k0;
            double s = 0.0;
            for (int l = 0; l < nb; ++l) s += row[l] * x[k0 + l];
            x[i] -= s;
        }
        __syncthreads();
    }
}

// L^T x = b in place (x holds b), one workgroup
__global__ __launch_bounds__(kBlock) void k_trsv_upper_t(const double* L, int32_t m, double* x) {
    const int lane = threadIdx.x;
    const int32_t nblk = (m + kNb - 1) / kNb;
    for (int32_t kb = nblk - 1; kb >= 0; --kb) {
        const int32_t k0 = kb * kNb;
        const int nb = min(kNb, m - k0);
        if (threadIdx.x < kWave) {
            double xi = lane < nb ? x[k0 + lane] : 0.0, mine = 0.0;
            for (int j = nb - 1; j >= 0; --j) {
                const double xj = __shfl(xi, j, kWave) / L[(int64_t)(k0 + j) * m + k0 + j];
                if (lane == j) mine = xj;
                if (lane < j) xi -= L[(int64_t)(k0 + j) * m + k0 + lane] * xj;
            }
            if (lane < nb) x[k0 + lane] = mine;
        }
        __syncthreads();
        for (int64_t i = threadIdx.x; i < k0; i += kBlock) {
            double s = 0.0;
            for (int l = 0; l < nb; ++l) s += L[(int64_t)(k0 + l) * m + i] * x[k0 + l];
            x[i] -= s;
        }
        __syncthreads();
    }
}

// --- per-iteration vector work
// d = x / z, r_xz (mode 0: -x z; 1: sigma_mu - x z - dxa dza), t = r_xz / z - d r_c
__global__ void k_ipm_t(const double* x, const double* z, const double* r_c, int mode, double sigma_mu,
                        const double* dxa, const double* dza, int64_t n, double* d, double* t) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const double dj = x[j] / z[j];
        const double rxz = mode == 0 ? -x[j] * z[j] : sigma_mu - x[j] * z[j] - dxa[j] * dza[j];
        d[j] = dj;
        t[j] = rxz / z[j] - dj * r_c[j];
    }
}

// dx = d v + t, dz = r_c - v
__global__ void k_ipm_dir(const double* d, const double* v, const double* t, const double* r_c, int64_t n,
                          double* dx, double* dz) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        dx[j] = d[j] * v[j] + t[j];
        dz[j] = r_c[j] - v[j];
    }
}

// fixed-order block partials: W quantities per block, then one workgroup
// combines them (sum, or min for the ratio tests)
template <int W>
__device__ void block_partials(double (&v)[W], bool minimum, double* out) {
    __shared__ double sh[W][kBlock];
#pragma unroll
    for (int q = 0; q < W; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st)
#pragma unroll
            for (int q = 0; q < W; ++q)
                sh[q][threadIdx.x] = minimum ? fmin(sh[q][threadIdx.x], sh[q][threadIdx.x + st])
                                             : sh[q][threadIdx.x] + sh[q][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < W) out[(int64_t)blockIdx.x * W + threadIdx.x] = sh[threadIdx.x][0];
}

// step to the boundary: min over dv < 0 of -v / dv, for (x, dx) and (z, dz)
__global__ __launch_bounds__(kBlock) void k_ipm_ratio(const double* x, const double* dx, const double* z,
                                                      const double* dz, int64_t n, double* part) {
    double v[2] = {INFINITY, INFINITY};
    for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        if (dx[j] < 0.0) v[0] = fmin(v[0], -x[j] / dx[j]);
        if (dz[j] < 0.0) v[1] = fmin(v[1], -z[j] / dz[j]);
    }
    block_partials<2>(v, true, part);
}

// sum (x + ap dx)(z + ad dz)
__global__ __launch_bounds__(kBlock) void k_ipm_mu_at(const double* x, const double* dx, const double* z,
                                                      const double* dz, int64_t n, const double* steps,
                                                      double* part) {
    const double ap = steps[0], ad = steps[1];
    double v[1] = {0.0};
    for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock)
        v[0] += (x[j] + ap * dx[j]) * (z[j] + ad * dz[j]);
    block_partials<1>(v, false, part);
}

// ||r_c||^2, c~^T x, x^T z over n; ||r_b||^2, b~^T y over m (two launches)
__global__ __launch_bounds__(kBlock) void k_ipm_sums3(const double* a, const double* b, const double* c,
                                                      const double* d, int64_t n, double* part) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        v[0] += a[j] * a[j];
        v[1] += b[j] * c[j];
        if (d) v[2] += c[j] * d[j];
    }
    block_partials<3>(v, false, part);
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_ipm_final(const double* part, int G, int minimum_mask, double* out) {
    __shared__ double sh[kBlock];
    for (int q = 0; q < W; ++q) {
        const bool mn = (minimum_mask >> q) & 1;
        double s = mn ? INFINITY : 0.0;
        for (int g = threadIdx.x; g < G; g += kBlock) {
            const double v = part[(int64_t)g * W + q];
            s = mn ? fmin(s, v) : s + v;
        }
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int st = kBlock / 2; st > 0; st >>= 1) {
            if (threadIdx.x < st)
                sh[threadIdx.x] = mn ? fmin(sh[threadIdx.x], sh[threadIdx.x + st]) : sh[threadIdx.x] + sh[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[q] = sh[0];
        __syncthreads();
    }
}

// v += a s .* dv for up to three (vector, direction, step slot) triples
__global__ void k_ipm_step(double* x, const double* dx, int64_t n, double* y, const double* dy, int64_t m, double* z,
                           const double* dz, const double* steps) {
    const double ap = steps[0], ad = steps[1];
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        x[j] = x[j] + ap * dx[j];
        z[j] = z[j] + ad * dz[j];
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = y[i] + ad * dy[i];
}

__global__ void k_zero_flag(int32_t* f) {
    if (threadIdx.x < 4) f[threadIdx.x] = 0;
}

// v + s for Mehrotra's shifts
__global__ void k_ipm_shift(double* v, int64_t n, double s) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        v[j] = v[j] + s;
}

// sum and min of a vector, and its dot with another: part[g] = {sum a, min a, sum a b}
__global__ __launch_bounds__(kBlock) void k_ipm_summin(const double* a, const double* b, int64_t n, double* part) {
    double v[3] = {0.0, INFINITY, 0.0};
    for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        v[0] += a[j];
        v[1] = fmin(v[1], a[j]);
        if (b) v[2] += a[j] * b[j];
    }
    // min needs its own combine: reuse block_partials twice
    double s[2] = {v[0], v[2]};
    double mn[1] = {v[1]};
    block_partials<2>(s, false, part);
    __syncthreads();
    block_partials<1>(mn, true, part + 2 * (int64_t)gridDim.x);
}

struct IpmWs {
    double *M, *av, *atv, *bt, *ct, *x, *y, *z, *dx, *dy, *dz, *dxa, *dya, *dza, *d, *t, *v, *rb, *rc, *rhs;
    double *xc, *yc, *zc, *part, *scal;
    int32_t* flag;
    void* cws;  // centering workspace
    size_t bytes;
};

IpmWs carve_ipm(void* base, int64_t m, int64_t n, int64_t nnz) {
    Carver cv(base, 0);
    IpmWs w;
    w.M = cv.take<double>((size_t)(m * m));
    w.av = cv.take<double>(nnz);
    w.atv = cv.take<double>(nnz);
    w.bt = cv.take<double>(m);
    w.ct = cv.take<double>(n);
    w.x = cv.take<double>(n);
    w.y = cv.take<double>(m);
    w.z = cv.take<double>(n);
    w.dx = cv.take<double>(n);
    w.dy = cv.take<double>(m);
    w.dz = cv.take<double>(n);
    w.dxa = cv.take<double>(n);
    w.dya = cv.take<double>(m);
    w.dza = cv.take<double>(n);
    w.d = cv.take<double>(n);
    w.t = cv.take<double>(n);
    w.v = cv.take<double>(std::max(m, n));
    w.rb = cv.take<double>(m);
    w.rc = cv.take<double>(n);
    w.rhs = cv.take<double>(m);
    w.xc = cv.take<double>(n);
    w.yc = cv.take<double>(m);
    w.zc = cv.take<double>(n);
    w.part = cv.take<double>((size_t)kRedBlocks * 4);
    w.scal = cv.take<double>(16);
    w.flag = cv.take<int32_t>(4);
    w.cws = cv.take<char>(mipdhg_center_workspace_size((int32_t)n));
    w.bytes = cv.off;
    return w;
}

int red_grid(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(kRedBlocks, (n + kBlock - 1) / kBlock)); }
int rows_grid(int64_t rows) { return (int)((rows + kBlock / kWave - 1) / (kBlock / kWave)); }

struct Ipm {
    const mipdhg_lp& lp;
    const mipdhg_ipm_options& o;
    hipStream_t s;
    IpmWs w;
    int64_t m, n;
    int pivots = 0;

    int spmv_a(const double* v, const double* s0, double sgn, const double* s1, double* out) {
        hipLaunchKernelGGL(k_ipm_spmv, dim3(rows_grid(m)), dim3(kBlock), 0, s, lp.a_rowptr, lp.a_col,
                           (const double*)w.av, v, (int32_t)m, s0, sgn, s1, out);
        MIP_LAUNCH_CHECK();
        return 0;
    }
    int spmv_at(const double* v, const double* s0, double sgn, const double* s1, double* out) {
        hipLaunchKernelGGL(k_ipm_spmv, dim3(rows_grid(n)), dim3(kBlock), 0, s, lp.at_rowptr, lp.at_col,
                           (const double*)w.atv, v, (int32_t)n, s0, sgn, s1, out);
        MIP_LAUNCH_CHECK();
        return 0;
    }
    // M = A~ diag(wt) A~^T (lower), then its Cholesky factor in place
    int factor(const double* wt) {
        hipLaunchKernelGGL(k_ipm_normal, dim3((unsigned)((m + kBlock - 1) / kBlock), (unsigned)m), dim3(kBlock), 0, s,
                           lp.a_rowptr, lp.a_col, (const double*)w.av, wt, (int32_t)m, w.M);
        MIP_LAUNCH_CHECK();
        for (int64_t k0 = 0; k0 < m; k0 += kNb) {
            const int nb = (int)std::min<int64_t>(kNb, m - k0);
            hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(kBlock), 0, s, w.M, (int32_t)m, (int32_t)k0, nb, w.flag);
            const int64_t rest = m - k0 - nb;
            if (rest > 0) {
                hipLaunchKernelGGL(k_chol_panel, dim3((unsigned)((rest + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                                   w.M, (int32_t)m, (int32_t)k0, nb);
                const int64_t T = (rest + kNb - 1) / kNb;
                hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(T * (T + 1) / 2)), dim3(kBlock), 0, s, w.M,
                                   (int32_t)m, (int32_t)k0, nb);
            }
            MIP_LAUNCH_CHECK();
        }
        return 0;
    }
    // x <- M^-1 x with the factor in M
    int solve(double* x) {
        hipLaunchKernelGGL(k_trsv_lower, dim3(1), dim3(kBlock), 0, s, (const double*)w.M, (int32_t)m, x);
        hipLaunchKernelGGL(k_trsv_upper_t, dim3(1), dim3(kBlock), 0, s, (const double*)w.M, (int32_t)m, x);
        MIP_LAUNCH_CHECK();
        return 0;
    }
    template <int W>
    int reduce(int64_t len, int G, int minmask, double* host) {
        hipLaunchKernelGGL((k_ipm_final<W>), dim3(1), dim3(kBlock), 0, s, (const double*)w.part, G, minmask, w.scal);
        MIP_LAUNCH_CHECK();
        MIP_HIP(hipMemcpyAsync(host, w.scal, W * sizeof(double), hipMemcpyDeviceToHost, s));
        MIP_HIP(hipStreamSynchronize(s));
        (void)len;
        return 0;
    }

    // Mehrotra's start: x = A~^T (A~ A~^T)^-1 b~, y = (A~ A~^T)^-1 A~ c~,
    // z = c~ - A~^T y, shifted by max(-1.5 min, 0), then by half of x^T z
    // over the sum of the other vector
    int cold_start() {
        int rc;
        if ((rc = factor(nullptr))) return rc;
        MIP_HIP(hipMemcpyAsync(w.rhs, w.bt, m * 8, hipMemcpyDeviceToDevice, s));
        if ((rc = solve(w.rhs))) return rc;
        if ((rc = spmv_at(w.rhs, nullptr, 1.0, nullptr, w.x))) return rc;
        if ((rc = spmv_a(w.ct, nullptr, 1.0, nullptr, w.y))) return rc;
        if ((rc = solve(w.y))) return rc;
        if ((rc = spmv_at(w.y, w.ct, -1.0, nullptr, w.z))) return rc;
        const int G = red_grid(n);
        double hx[3], hz[3];
        hipLaunchKernelGGL(k_ipm_summin, dim3(G), dim3(kBlock), 0, s, (const double*)w.x, (const double*)nullptr, n,
                           w.part);
        MIP_LAUNCH_CHECK();
        if ((rc = finish_summin(G, hx))) return rc;
        hipLaunchKernelGGL(k_ipm_summin, dim3(G), dim3(kBlock), 0, s, (const double*)w.z, (const double*)nullptr, n,
                           w.part);
        MIP_LAUNCH_CHECK();
        if ((rc = finish_summin(G, hz))) return rc;
        const double sx = std::max(-1.5 * hx[1], 0.0), sz = std::max(-1.5 * hz[1], 0.0);
        hipLaunchKernelGGL(k_ipm_shift, dim3(grid_for(n)), dim3(kBlock), 0, s, w.x, n, sx);
        hipLaunchKernelGGL(k_ipm_shift, dim3(grid_for(n)), dim3(kBlock), 0, s, w.z, n, sz);
        MIP_LAUNCH_CHECK();
        // x^T z, sum x, sum z of the shifted vectors
        hipLaunchKernelGGL(k_ipm_summin, dim3(G), dim3(kBlock), 0, s, (const double*)w.x, (const double*)w.z, n,
                           w.part);
        MIP_LAUNCH_CHECK();
        if ((rc = finish_summin(G, hx))) return rc;
        hipLaunchKernelGGL(k_ipm_summin, dim3(G), dim3(kBlock), 0, s, (const double*)w.z, (const double*)nullptr, n,
                           w.part);
        MIP_LAUNCH_CHECK();
        if ((rc = finish_summin(G, hz))) return rc;
        const double xz = hx[2];
        hipLaunchKernelGGL(k_ipm_shift, dim3(grid_for(n)), dim3(kBlock), 0, s, w.x, n, 0.5 * xz / hz[0]);
        hipLaunchKernelGGL(k_ipm_shift, dim3(grid_for(n)), dim3(kBlock), 0, s, w.z, n, 0.5 * xz / hx[0]);
        MIP_LAUNCH_CHECK();
        return 0;
    }
    // {sum a, min a, sum a b} from k_ipm_summin's partials
    int finish_summin(int G, double* h) {
        double s2[2], s1[1];
        hipLaunchKernelGGL((k_ipm_final<2>), dim3(1), dim3(kBlock), 0, s, (const double*)w.part, G, 0, w.scal);
        hipLaunchKernelGGL((k_ipm_final<1>), dim3(1), dim3(kBlock), 0, s, (const double*)(w.part + 2 * G), G, 1,
                           w.scal + 2);
        MIP_LAUNCH_CHECK();
        MIP_HIP(hipMemcpyAsync(s2, w.scal, 2 * 8, hipMemcpyDeviceToHost, s));
        MIP_HIP(hipMemcpyAsync(s1, w.scal + 2, 8, hipMemcpyDeviceToHost, s));
        MIP_HIP(hipStreamSynchronize(s));
        h[0] = s2[0];
        h[1] = s1[0];
        h[2] = s2[1];
        return 0;
    }

    // the relative measures (rp, rd, gap) and c~^T x, b~^T y, x^T z; r_b, r_c left in the workspace
    int measures(double* rel, double* px, double* dy, double* xz) {
        int rc;
        if ((rc = spmv_a(w.x, w.bt, -1.0, nullptr, w.rb))) return rc;
        if ((rc = spmv_at(w.y, w.ct, -1.0, w.z, w.rc))) return rc;
        double hn[3], hm[3];
        int G = red_grid(n);
        hipLaunchKernelGGL(k_ipm_sums3, dim3(G), dim3(kBlock), 0, s, (const double*)w.rc, (const double*)w.ct,
                           (const double*)w.x, (const double*)w.z, n, w.part);
        MIP_LAUNCH_CHECK();
        if ((rc = reduce<3>(n, G, 0, hn))) return rc;
        G = red_grid(m);
        hipLaunchKernelGGL(k_ipm_sums3, dim3(G), dim3(kBlock), 0, s, (const double*)w.rb, (const double*)w.bt,
                           (const double*)w.y, (const double*)nullptr, m, w.part);
        MIP_LAUNCH_CHECK();
        if ((rc = reduce<3>(m, G, 0, hm))) return rc;
        rel[0] = sqrt(hm[0]) / (1.0 + bnorm);
        rel[1] = sqrt(hn[0]) / (1.0 + cnorm);
        *px = hn[1];
        *dy = hm[1];
        *xz = hn[2];
        rel[2] = fabs(*px - *dy) / (1.0 + fabs(*px) + fabs(*dy));
        return 0;
    }
    double bnorm = 0.0, cnorm = 0.0;

    // direction for r_xz of `mode` (see k_ipm_t) into (dx, dy, dz)
    int direction(int mode, double sigma_mu, double* dx, double* dy, double* dz) {
        int rc;
        hipLaunchKernelGGL(k_ipm_t, dim3(grid_for(n)), dim3(kBlock), 0, s, (const double*)w.x, (const double*)w.z,
                           (const double*)w.rc, mode, sigma_mu, (const double*)w.dxa, (const double*)w.dza, n, w.d,
                           w.t);
        MIP_LAUNCH_CHECK();
        if ((rc = spmv_a(w.t, w.rb, -1.0, nullptr, dy))) return rc;  // r_b - A~ t
        if ((rc = solve(dy))) return rc;
        if ((rc = spmv_at(dy, nullptr, 1.0, nullptr, w.v))) return rc;
        hipLaunchKernelGGL(k_ipm_dir, dim3(grid_for(n)), dim3(kBlock), 0, s, (const double*)w.d, (const double*)w.v,
                           (const double*)w.t, (const double*)w.rc, n, dx, dz);
        MIP_LAUNCH_CHECK();
        return 0;
    }
    // steps to the boundary of (x, dx) and (z, dz)
    int boundary(const double* dx, const double* dz, double* h) {
        const int G = red_grid(n);
        hipLaunchKernelGGL(k_ipm_ratio, dim3(G), dim3(kBlock), 0, s, (const double*)w.x, dx, (const double*)w.z, dz,
                           n, w.part);
        MIP_LAUNCH_CHECK();
        return reduce<2>(n, G, 3, h);
    }

    // the iteration from the point in (x, y, z); fills info
    int run(mipdhg_ipm_info* info) {
        int rc;
        info->iters = 0;
        info->status = MIPDHG_ITER_LIMIT;
        for (int k = 0;; ++k) {
            double rel[3], px, dyv, xz;
            if ((rc = measures(rel, &px, &dyv, &xz))) return rc;
            info->rel_rp = rel[0];
            info->rel_rd = rel[1];
            info->rel_gap = rel[2];
            if (!(std::isfinite(rel[0]) && std::isfinite(rel[1]) && std::isfinite(rel[2]))) {
                info->status = MIPDHG_NUMERICAL;
                break;
            }
            if (std::max(rel[0], std::max(rel[1], rel[2])) <= o.tol) {
                info->status = MIPDHG_OPTIMAL;
                break;
            }
            if (k == o.max_iter) break;
            const double mu = xz / (double)n;
            hipLaunchKernelGGL(k_ipm_vscale, dim3(grid_for(n)), dim3(kBlock), 0, s, (const double*)w.x,
                               (const double*)w.z, 1, n, w.d);  // D = X Z^-1
            MIP_LAUNCH_CHECK();
            if ((rc = factor(w.d))) return rc;
            // predictor
            if ((rc = direction(0, 0.0, w.dxa, w.dya, w.dza))) return rc;
            double st[2];
            if ((rc = boundary(w.dxa, w.dza, st))) return rc;
            double steps[2] = {std::min(1.0, st[0]), std::min(1.0, st[1])};
            MIP_HIP(hipMemcpyAsync(w.scal + 8, steps, 16, hipMemcpyHostToDevice, s));
            MIP_HIP(hipStreamSynchronize(s));
            const int G = red_grid(n);
            hipLaunchKernelGGL(k_ipm_mu_at, dim3(G), dim3(kBlock), 0, s, (const double*)w.x, (const double*)w.dxa,
                               (const double*)w.z, (const double*)w.dza, n, (const double*)(w.scal + 8), w.part);
            MIP_LAUNCH_CHECK();
            double mua[1];
            if ((rc = reduce<1>(n, G, 0, mua))) return rc;
            const double sigma = std::pow((mua[0] / (double)n) / mu, 3.0);
            // corrector, with the same factor
            if ((rc = direction(1, sigma * mu, w.dx, w.dy, w.dz))) return rc;
            if ((rc = boundary(w.dx, w.dz, st))) return rc;
            steps[0] = std::min(1.0, o.step_frac * st[0]);
            steps[1] = std::min(1.0, o.step_frac * st[1]);
            if (k == 0) {
                info->first_step_p = steps[0];
                info->first_step_d = steps[1];
            }
            MIP_HIP(hipMemcpyAsync(w.scal + 8, steps, 16, hipMemcpyHostToDevice, s));
            MIP_HIP(hipStreamSynchronize(s));
            hipLaunchKernelGGL(k_ipm_step, dim3(grid_for(std::max(m, n))), dim3(kBlock), 0, s, w.x,
                               (const double*)w.dx, n, w.y, (const double*)w.dy, m, w.z, (const double*)w.dz,
                               (const double*)(w.scal + 8));
            MIP_LAUNCH_CHECK();
            info->iters = k + 1;
        }
        return 0;
    }
};

}  // namespace
}  // namespace mip

using namespace mip;

namespace {

int check_ipm(const mipdhg_lp* lp, const mipdhg_ipm_options* o) {
    int rc = check_lp(lp);
    if (rc) return rc;
    if (!o) return set_error("options are NULL"), MIPDHG_ERR_INVALID_ARG;
    if (lp->lo || lp->hi || lp->sense)
        return set_error("the interior-point consumer takes the standard form"), MIPDHG_ERR_UNSUPPORTED;
    if (lp->m > kIpmMaxM)
        return set_error("m = %d: the dense normal matrix is limited to m <= %d", lp->m, kIpmMaxM),
               MIPDHG_ERR_UNSUPPORTED;
    if (!(o->tol > 0.0) || o->max_iter < 0 || !(o->step_frac > 0.0 && o->step_frac < 1.0) || !(o->min_step >= 0.0) ||
        o->max_lifts < 0 || !(o->mu_min >= 0.0) || !(o->delta_max >= 0.0) || !(o->alpha_min > 0.0) ||
        !std::isfinite(o->tol) || !std::isfinite(o->alpha_min) || !std::isfinite(o->mu_min) ||
        !std::isfinite(o->delta_max))
        return set_error("ipm options: tol > 0, max_iter >= 0, 0 < step_frac < 1, min_step >= 0, max_lifts >= 0, "
                         "mu_min >= 0, delta_max >= 0, alpha_min > 0, all finite"),
               MIPDHG_ERR_INVALID_ARG;
    return 0;
}

// the scaled LP in the workspace, after checking that A's rows are sorted
int ipm_setup(Ipm& P, const double* d_row, const double* d_col) {
    const mipdhg_lp& lp = P.lp;
    hipStream_t s = P.s;
    std::vector<int32_t> rp(lp.m + 1), col(lp.nnz);
    MIP_HIP(hipMemcpyAsync(rp.data(), lp.a_rowptr, rp.size() * 4, hipMemcpyDeviceToHost, s));
    if (lp.nnz) MIP_HIP(hipMemcpyAsync(col.data(), lp.a_col, col.size() * 4, hipMemcpyDeviceToHost, s));
    MIP_HIP(hipStreamSynchronize(s));
    int rc = check_rowptr(rp, lp.m, lp.nnz, "A");
    if (rc) return rc;
    for (int32_t r = 0; r < lp.m; ++r)
        for (int32_t k = rp[r]; k < rp[r + 1]; ++k) {
            if (col[k] < 0 || col[k] >= lp.n)
                return set_error("A: column index out of range in row %d", r), MIPDHG_ERR_BAD_CSR;
            if (k > rp[r] && col[k] <= col[k - 1])
                return set_error("A: the interior-point consumer needs each row's columns strictly increasing "
                                 "(row %d)", r),
                       MIPDHG_ERR_BAD_CSR;
        }
    const IpmWs& w = P.w;
    hipLaunchKernelGGL(k_ipm_scale_vals, dim3(grid_for(lp.m)), dim3(kBlock), 0, s, lp.a_rowptr, lp.a_col, lp.a_val,
                       lp.m, d_row, d_col, 0, w.av);
    hipLaunchKernelGGL(k_ipm_scale_vals, dim3(grid_for(lp.n)), dim3(kBlock), 0, s, lp.at_rowptr, lp.at_col, lp.at_val,
                       lp.n, d_row, d_col, 1, w.atv);
    hipLaunchKernelGGL(k_ipm_vscale, dim3(grid_for(lp.m)), dim3(kBlock), 0, s, lp.b, d_row, 0, (int64_t)lp.m, w.bt);
    hipLaunchKernelGGL(k_ipm_vscale, dim3(grid_for(lp.n)), dim3(kBlock), 0, s, lp.c, d_col, 0, (int64_t)lp.n, w.ct);
    hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(32), 0, s, w.flag);
    MIP_LAUNCH_CHECK();
    double hb[3], hc[3];
    int G = red_grid(lp.m);
    hipLaunchKernelGGL(k_ipm_sums3, dim3(G), dim3(kBlock), 0, s, (const double*)w.bt, (const double*)w.bt,
                       (const double*)w.bt, (const double*)nullptr, (int64_t)lp.m, w.part);
    MIP_LAUNCH_CHECK();
    if ((rc = P.reduce<3>(lp.m, G, 0, hb))) return rc;
    G = red_grid(lp.n);
    hipLaunchKernelGGL(k_ipm_sums3, dim3(G), dim3(kBlock), 0, s, (const double*)w.ct, (const double*)w.ct,
                       (const double*)w.ct, (const double*)nullptr, (int64_t)lp.n, w.part);
    MIP_LAUNCH_CHECK();
    if ((rc = P.reduce<3>(lp.n, G, 0, hc))) return rc;
    P.bnorm = sqrt(hb[0]);
    P.cnorm = sqrt(hc[0]);
    return 0;
}

// the point in the workspace, unscaled into the outputs; objectives and pivots into info
int ipm_finish(Ipm& P, const double* d_row, const double* d_col, double* x, double* y, double* z,
               mipdhg_ipm_info* info) {
    hipStream_t s = P.s;
    const IpmWs& w = P.w;
    hipLaunchKernelGGL(k_ipm_vscale, dim3(grid_for(P.n)), dim3(kBlock), 0, s, (const double*)w.x, d_col, 0, P.n, x);
    hipLaunchKernelGGL(k_ipm_vscale, dim3(grid_for(P.m)), dim3(kBlock), 0, s, (const double*)w.y, d_row, 0, P.m, y);
    hipLaunchKernelGGL(k_ipm_vscale, dim3(grid_for(P.n)), dim3(kBlock), 0, s, (const double*)w.z, d_col, 1, P.n, z);
    MIP_LAUNCH_CHECK();
    double rel[3], px, dy, xz;
    int rc = P.measures(rel, &px, &dy, &xz);
    if (rc) return rc;
    int32_t piv = 0;
    MIP_HIP(hipMemcpyAsync(&piv, w.flag, 4, hipMemcpyDeviceToHost, s));
    MIP_HIP(hipStreamSynchronize(s));
    info->pobj = px;
    info->dobj = dy;
    info->mu = xz / (double)P.n;
    info->pivots_replaced = piv;
    return 0;
}

}  // namespace

extern "C" void mipdhg_ipm_default_options(mipdhg_ipm_options* o) {
    if (!o) return;
    o->tol = 1e-8;
    o->max_iter = 100;
    o->step_frac = 0.9995;
    o->min_step = 1e-6;
    o->max_lifts = 12;
    o->mu_min = 1e-6;
    o->delta_max = 1e-4;
    o->alpha_min = 1e-6;
}

extern "C" int mipdhg_ipm_workspace_size(const mipdhg_lp* lp, size_t* bytes) {
    clear_error();
    if (!bytes) return set_error("bytes is NULL"), MIPDHG_ERR_INVALID_ARG;
    int rc = check_lp(lp);
    if (rc) return rc;
    if (lp->m > kIpmMaxM)
        return set_error("m = %d: the dense normal matrix is limited to m <= %d", lp->m, kIpmMaxM),
               MIPDHG_ERR_UNSUPPORTED;
    *bytes = carve_ipm(nullptr, lp->m, lp->n, lp->nnz).bytes;
    return 0;
}

extern "C" int mipdhg_ipm_solve(const mipdhg_lp* lp, const double* d_row, const double* d_col, const double* x_start,
                                const double* y_start, const double* z_start, const mipdhg_ipm_options* opt,
                                void* workspace, size_t workspace_bytes, void* stream, double* x, double* y, double* z,
                                mipdhg_ipm_info* info) {
    clear_error();
    int rc = check_ipm(lp, opt);
    if (rc) return rc;
    const bool cold = !x_start && !y_start && !z_start;
    if (!cold && !(x_start && y_start && z_start))
        return set_error("give all three of x_start, y_start, z_start or none"), MIPDHG_ERR_INVALID_ARG;
    if (!workspace || !x || !y || !z || !info) return set_error("workspace, outputs and info are required"),
                                                      MIPDHG_ERR_INVALID_ARG;
    if (((uintptr_t)workspace & 255) != 0) return set_error("workspace must be 256-byte aligned"), MIPDHG_ERR_INVALID_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    Ipm P{*lp, *opt, (hipStream_t)stream, carve_ipm(workspace, lp->m, lp->n, lp->nnz), lp->m, lp->n};
    if (P.w.bytes > workspace_bytes)
        return set_error("workspace too small: %zu bytes given, %zu needed", workspace_bytes, P.w.bytes),
               MIPDHG_ERR_WORKSPACE;
    memset(info, 0, sizeof(*info));
    if ((rc = ipm_setup(P, d_row, d_col))) return rc;
    if (cold) {
        if ((rc = P.cold_start())) return rc;
    } else {
        MIP_HIP(hipMemcpyAsync(P.w.x, x_start, P.n * 8, hipMemcpyDeviceToDevice, P.s));
        MIP_HIP(hipMemcpyAsync(P.w.y, y_start, P.m * 8, hipMemcpyDeviceToDevice, P.s));
        MIP_HIP(hipMemcpyAsync(P.w.z, z_start, P.n * 8, hipMemcpyDeviceToDevice, P.s));
    }
    if ((rc = P.run(info))) return rc;
    if ((rc = ipm_finish(P, d_row, d_col, x, y, z, info))) return rc;
    info->alpha_min = 0.0;
    info->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return info->status;
}

extern "C" int mipdhg_ipm_warm(const mipdhg_lp* lp, const double* d_row, const double* d_col, const double* x_pdhg,
                               const double* y_pdhg, const double* z_pdhg, const mipdhg_ipm_options* opt,
                               void* workspace, size_t workspace_bytes, void* stream, double* x, double* y, double* z,
                               mipdhg_ipm_info* info) {
    clear_error();
    int rc = check_ipm(lp, opt);
    if (rc) return rc;
    if (!x_pdhg || !y_pdhg || !z_pdhg || !workspace || !x || !y || !z || !info)
        return set_error("the PDHG point, workspace, outputs and info are required"), MIPDHG_ERR_INVALID_ARG;
    if (((uintptr_t)workspace & 255) != 0) return set_error("workspace must be 256-byte aligned"), MIPDHG_ERR_INVALID_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    Ipm P{*lp, *opt, (hipStream_t)stream, carve_ipm(workspace, lp->m, lp->n, lp->nnz), lp->m, lp->n};
    if (P.w.bytes > workspace_bytes)
        return set_error("workspace too small: %zu bytes given, %zu needed", workspace_bytes, P.w.bytes),
               MIPDHG_ERR_WORKSPACE;
    memset(info, 0, sizeof(*info));
    if ((rc = ipm_setup(P, d_row, d_col))) return rc;
    // Algorithm 1 on the scaled point (x / D_c, y / D_r, z D_c)
    double mu_t = 0.0;
    if ((rc = mipdhg_center_start(lp->n, x_pdhg, z_pdhg, d_col, opt->mu_min, opt->delta_max, opt->alpha_min, P.w.cws,
                                  mipdhg_center_workspace_size(lp->n), stream, P.w.xc, P.w.zc, &mu_t)))
        return rc;
    hipLaunchKernelGGL(k_ipm_vscale, dim3(grid_for(P.m)), dim3(kBlock), 0, P.s, y_pdhg, d_row, 1, P.m, P.w.yc);
    MIP_LAUNCH_CHECK();
    double alpha = opt->alpha_min;
    int lifts = 0;
    while (true) {
        MIP_HIP(hipMemcpyAsync(P.w.x, P.w.xc, P.n * 8, hipMemcpyDeviceToDevice, P.s));
        MIP_HIP(hipMemcpyAsync(P.w.y, P.w.yc, P.m * 8, hipMemcpyDeviceToDevice, P.s));
        MIP_HIP(hipMemcpyAsync(P.w.z, P.w.zc, P.n * 8, hipMemcpyDeviceToDevice, P.s));
        if ((rc = P.run(info))) return rc;
        const bool small = info->iters >= 1 && std::min(info->first_step_p, info->first_step_d) < opt->min_step;
        if (!small || lifts >= opt->max_lifts) break;
        alpha *= 10.0;
        ++lifts;
        if ((rc = mipdhg_center_reclamp(lp->n, alpha, stream, P.w.xc, P.w.zc))) return rc;
    }
    if ((rc = ipm_finish(P, d_row, d_col, x, y, z, info))) return rc;
    info->lifts = lifts;
    info->alpha_min = alpha;
    info->mu_target = mu_t;
    info->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return info->status;
}
