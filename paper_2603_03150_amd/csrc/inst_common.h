// Per-instance pieces shared by the batched solve and the unrolled map: a
// fixed-order workgroup reduction and the instance set-up (norms, scaling,
// scaled values, power iteration, step and initial primal weight).
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace mip {

// Dot product of the sparse row [s, e) with a vector held in LDS, indexed by
// the instance-local column (16 bits: an instance's vectors fit in LDS, so
// its rows and columns number fewer than 65,536): the loads of four nonzeros
// are issued together, and the terms are added in the row's order.
template <typename Acc, typename V, typename X>
__device__ __forceinline__ Acc row_dot4(const V* vals, const uint16_t* cols, const X* xl, int s, int e) {
    Acc acc = 0;
    int k = s;
    for (; k + 4 <= e; k += 4) {
        int c[4];
        Acc v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            c[q] = cols[k + q];
            v[q] = (Acc)ld_val_cached(vals, k + q);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) acc += v[q] * (Acc)xl[c[q]];
    }
    for (; k < e; ++k) acc += (Acc)ld_val_cached(vals, k) * (Acc)xl[cols[k]];
    return acc;
}

// Largest instance dimension the 16-bit local columns address.
constexpr int kInstMaxDim = 65535;

constexpr int kBatchBlock = 256;

// Fixed-order workgroup sums (NS) and maxima (NM) over a workgroup of BS
// threads; every thread gets the result.  sh holds (NS + NM) * BS / 64 doubles.
template <int NS, int NM, int BS = kBatchBlock>
__device__ __forceinline__ void wg_reduce(double (&s)[NS > 0 ? NS : 1], double (&mx)[NM > 0 ? NM : 1],
                                          double* sh) {
    constexpr int NW = BS / kWave;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const double v = group_sum<kWave>(s[q]);
        if (lane == 0) sh[q * NW + wave] = v;
    }
#pragma unroll
    for (int q = 0; q < NM; ++q) {
        double v = mx[q];
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
        if (lane == 0) sh[(NS + q) * NW + wave] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        double v = sh[q * NW];
        for (int w = 1; w < NW; ++w) v += sh[q * NW + w];
        s[q] = v;
    }
#pragma unroll
    for (int q = 0; q < NM; ++q) {
        double v = sh[(NS + q) * NW];
        for (int w = 1; w < NW; ++w) v = fmax(v, sh[(NS + q) * NW + w]);
        mx[q] = v;
    }
    __syncthreads();
}

struct InstMat {  // the caller's float64 block-diagonal LP
    const int32_t *a_rowptr, *a_col;
    const double* a_val;
    const int32_t *at_rowptr, *at_col;
    const double* at_val;
    const double *b, *c;
};

struct InstSetup {
    double b_norm, c_norm, sigma_hat, eta, omega0;
};

// Instance rows [r0, r1), columns [c0, c1), set up by a workgroup of BS
// threads.  Writes D_r, D_c (float64), the
// scaled values of the instance's entries of A and A^T (type V) with their
// instance-local columns (a_cl: col - c0, at_cl: row - r0), b~ and c~ (type T),
// and returns the norms, sigma_hat, eta and omega_0.  pu, pav are float64
// scratch vectors indexed like x, y; xl[n] and yl[m] are LDS vectors of the
// workgroup, free during the set-up.
template <typename T, typename V, int BS = kBatchBlock>
__device__ InstSetup inst_setup(const InstMat& M, int r0, int r1, int c0, int c1, double* d_row, double* d_col,
                                double* pu, double* pav, V* a_vs, V* at_vs, uint16_t* a_cl,
                                uint16_t* at_cl, T* bt, T* ct, int ruiz, int pc, int power_iters,
                                double step_safety, T* xl, T* yl, double* sh) {
    const int tid = threadIdx.x;
    const int m = r1 - r0, n = c1 - c0;
    double nn[2] = {0.0, 0.0}, nomax[1] = {0.0};

    // norms of b and c
    for (int i = tid; i < m; i += BS) nn[0] += M.b[r0 + i] * M.b[r0 + i];
    for (int j = tid; j < n; j += BS) nn[1] += M.c[c0 + j] * M.c[c0 + j];
    wg_reduce<2, 0, BS>(nn, nomax, sh);
    const double b_norm = sqrt(nn[0]), c_norm = sqrt(nn[1]);

    // scaling: Ruiz infinity-norm passes, then one Pock-Chambolle pass
    for (int i = tid; i < m; i += BS) d_row[r0 + i] = 1.0;
    for (int j = tid; j < n; j += BS) d_col[c0 + j] = 1.0;
    __syncthreads();
    const int passes = ruiz + (pc ? 1 : 0);
    double* stat_r = pav;
    double* stat_c = pu;
    for (int ps = 0; ps < passes; ++ps) {
        const bool mxm = ps < ruiz;
        for (int i = tid; i < m; i += BS) {
            const int g = r0 + i;
            double acc = 0.0;
            for (int k = M.a_rowptr[g]; k < M.a_rowptr[g + 1]; ++k) {
                const double v = fabs(M.a_val[k]) * d_col[M.a_col[k]];
                acc = mxm ? fmax(acc, v) : acc + v;
            }
            stat_r[g] = d_row[g] * acc;
        }
        for (int j = tid; j < n; j += BS) {
            const int g = c0 + j;
            double acc = 0.0;
            for (int k = M.at_rowptr[g]; k < M.at_rowptr[g + 1]; ++k) {
                const double v = fabs(M.at_val[k]) * d_row[M.at_col[k]];
                acc = mxm ? fmax(acc, v) : acc + v;
            }
            stat_c[g] = d_col[g] * acc;
        }
        __syncthreads();
        for (int i = tid; i < m; i += BS) {
            const double s = stat_r[r0 + i];
            if (s > 0.0) d_row[r0 + i] *= 1.0 / sqrt(s);
        }
        for (int j = tid; j < n; j += BS) {
            const double s = stat_c[c0 + j];
            if (s > 0.0) d_col[c0 + j] *= 1.0 / sqrt(s);
        }
        __syncthreads();
    }
    // scaled values in the iteration precision, b~ and c~ (norms in float64)
    double tn[2] = {0.0, 0.0};
    for (int i = tid; i < m; i += BS) {
        const int g = r0 + i;
        const double dr = d_row[g];
        for (int k = M.a_rowptr[g]; k < M.a_rowptr[g + 1]; ++k) {
            const int j = M.a_col[k];
            const double v = dr * M.a_val[k] * d_col[j];
            if constexpr (sizeof(V) == 2) a_vs[k] = f32_to_bf16_rne((float)v);
            else a_vs[k] = (V)v;
            a_cl[k] = (uint16_t)(j - c0);
        }
        const double btv = dr * M.b[g];
        bt[g] = (T)btv;
        tn[0] += btv * btv;
    }
    for (int j = tid; j < n; j += BS) {
        const int g = c0 + j;
        const double dc = d_col[g];
        for (int k = M.at_rowptr[g]; k < M.at_rowptr[g + 1]; ++k) {
            const int i = M.at_col[k];
            const double v = dc * M.at_val[k] * d_row[i];
            if constexpr (sizeof(V) == 2) at_vs[k] = f32_to_bf16_rne((float)v);
            else at_vs[k] = (V)v;
            at_cl[k] = (uint16_t)(i - r0);
        }
        const double ctv = dc * M.c[g];
        ct[g] = (T)ctv;
        tn[1] += ctv * ctv;
    }
    wg_reduce<2, 0, BS>(tn, nomax, sh);
    const double nbt = sqrt(tn[0]), nct = sqrt(tn[1]);

    // power iteration on the scaled iteration copy (the values and 16-bit
    // columns the iterations apply), as in the single-LP solve: vectors in
    // the iterate type, held in LDS (v in xl, A~ v in yl), products and sums
    // in float64.  u = A~^T (A~ v) overwrites v, which it no longer needs.
    __syncthreads();  // the scaled copies above are read by other threads
    for (int j = tid; j < n; j += BS) xl[j] = (T)(1.0 / sqrt((double)n));
    __syncthreads();
    double h = 0.0, h_m10 = 0.0;
    for (int kk = 0; kk <= power_iters; ++kk) {
        double s1[1] = {0.0};
        for (int i = tid; i < m; i += BS) {
            const int g = r0 + i;
            const double t = row_dot4<double>(a_vs, a_cl, xl, M.a_rowptr[g], M.a_rowptr[g + 1]);
            yl[i] = (T)t;
            s1[0] += t * t;
        }
        wg_reduce<1, 0, BS>(s1, nomax, sh);
        h = sqrt(s1[0]);
        if (kk == power_iters - 10) h_m10 = h;
        if (kk == power_iters) break;
        double s2[1] = {0.0};
        for (int j = tid; j < n; j += BS) {
            const int g = c0 + j;
            const double t = row_dot4<double>(at_vs, at_cl, yl, M.at_rowptr[g], M.at_rowptr[g + 1]);
            xl[j] = (T)t;
            s2[0] += t * t;
        }
        wg_reduce<1, 0, BS>(s2, nomax, sh);
        const double nu = sqrt(s2[0]);
        if (nu != 0.0)
            for (int j = tid; j < n; j += BS) xl[j] = (T)((double)xl[j] / nu);
        __syncthreads();
    }
    const double sigma_hat = h;
    double eta;
    if (sigma_hat <= 0.0) eta = step_safety;
    else if (pc && power_iters >= 10 && fabs(h - h_m10) > 1e-3 * h) eta = step_safety;
    else eta = step_safety / sigma_hat;
    const double omega0 = (nbt > 1e-10 && nct > 1e-10) ? nct / nbt : 1.0;
    InstSetup out;
    out.b_norm = b_norm;
    out.c_norm = c_norm;
    out.sigma_hat = sigma_hat;
    out.eta = eta;
    out.omega0 = omega0;
    return out;
}

}  // namespace mip
