// Input validation shared by the single and batched solves: column ranges,
// finiteness, and a dot-product test that A^T is the transpose of A.
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.h"
#include "plain.h"

namespace mip {

// flags: bit0 column index out of range, bit1 non-finite value, bit2 non-finite b/c
__global__ void k_check_entries(const int32_t* col, const double* val, int64_t nnz, int32_t ncols,
                                int32_t* flags) {
    int f = 0;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * blockDim.x) {
        int32_t j = col[k];
        if (j < 0 || j >= ncols) f |= 1;
        if (!isfinite(val[k])) f |= 2;
    }
    if (f) atomicOr(flags, f);
}

__global__ void k_check_vec(const double* v, int64_t n, int32_t* flags) {
    int f = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(v[i])) f |= 4;
    if (f) atomicOr(flags, f);
}

// general form: bit3 a bound is NaN, lo = +inf, hi = -inf or lo > hi;
// bit4 a row sense outside {0, 1, 2}
__global__ void k_check_bounds(const double* lo, const double* hi, int64_t n, int32_t* flags) {
    int f = 0;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const double l = lo ? lo[j] : 0.0, u = hi ? hi[j] : INFINITY;
        if (!(l <= u) || l == INFINITY || u == -INFINITY) f |= 8;  // NaN fails l <= u
    }
    if (f) atomicOr(flags, f);
}

__global__ void k_check_sense(const int8_t* sense, int64_t m, int32_t* flags) {
    int f = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        if (sense[i] < 0 || sense[i] > 2) f |= 16;
    if (f) atomicOr(flags, f);
}

__device__ __forceinline__ double hash_unit(uint32_t i, uint32_t seed) {
    uint32_t h = i * 0x9E3779B1u ^ seed;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return (double)h * (2.0 / 4294967296.0) - 1.0;  // [-1, 1)
}

// With u = hash(row), v = hash(col): partial sums of u_r (M v)_r (ABS = false)
// or of |u_r| sum_c |M_rc v_c| (ABS = true) over the rows of M.
template <bool ABS>
__global__ __launch_bounds__(kBlock) void k_transpose_dot(TilePlan p, const int32_t* col, const double* val,
                                                          uint32_t seed_row, uint32_t seed_col, double* partials) {
    extern __shared__ __align__(16) unsigned char smem_t[];
    const auto L = tile_lds<double>(smem_t, p);
    double s[1] = {0.0};
    double mx[1] = {0.0};
    auto prod = [&](int b, int j) {
        const int64_t k = (int64_t)b + j;
        const double t = val[k] * hash_unit((uint32_t)col[k], seed_col);
        return ABS ? fabs(t) : t;
    };
    auto epi = [&](int r, double t) {
        const double u = hash_unit((uint32_t)r, seed_row);
        s[0] += (ABS ? fabs(u) : u) * t;
    };
    auto le = lepi(epi);
    tiled_rows<false>(p, own_tile(), L, prod, le);
    block_reduce_store<1, 0>(s, mx, partials + blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_sum_partials(const double* partials, int G, double* out) {
    __shared__ double sh[kBlock];
    double s = 0.0;
    for (int g = threadIdx.x; g < G; g += kBlock) s += partials[g];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// Order-independent 64-bit hash of a column index array: the wrapping sum
// over k of a mix of (k, col[k]) (integer adds commute, so the result does
// not depend on the launch).
__device__ __forceinline__ uint64_t mix64(uint64_t v) {
    v ^= v >> 33;
    v *= 0xff51afd7ed558ccdull;
    v ^= v >> 33;
    v *= 0xc4ceb9fe1a85ec53ull;
    v ^= v >> 33;
    return v;
}

__global__ void k_hash_cols(const int32_t* col, int64_t nnz, unsigned long long* out) {
    uint64_t h = 0;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x)
        h += mix64(((uint64_t)k << 32) ^ (uint32_t)col[k]);
    for (int o = kWave / 2; o > 0; o >>= 1) h += __shfl_xor(h, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(out, (unsigned long long)h);
}

int column_hash(const int32_t* col, int64_t nnz, uint64_t* scratch, hipStream_t stream, uint64_t* out) {
    MIP_HIP(hipMemsetAsync(scratch, 0, 8, stream));
    if (nnz > 0)
        hipLaunchKernelGGL(k_hash_cols, dim3(grid_for(nnz)), dim3(kBlock), 0, stream, col, nnz,
                           (unsigned long long*)scratch);
    MIP_LAUNCH_CHECK();
    MIP_HIP(hipMemcpyAsync(out, scratch, 8, hipMemcpyDeviceToHost, stream));
    MIP_HIP(hipStreamSynchronize(stream));
    return 0;
}

int allow_validate_lds(int bytes) {
    if (bytes <= 65536) return 0;
    if (hipFuncSetAttribute((const void*)k_transpose_dot<false>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) !=
            hipSuccess ||
        hipFuncSetAttribute((const void*)k_transpose_dot<true>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) !=
            hipSuccess)
        return set_error("tile shape needs %d bytes of LDS per workgroup, more than the device allows", bytes),
               MIPDHG_ERR_UNSUPPORTED;
    return 0;
}

int validate_device(const mipdhg_lp& lp, const TilePlan& ta, const TilePlan& tat, int32_t* flags,
                    double* partials, double* red, hipStream_t stream) {
    const int64_t nnz = lp.nnz;
    MIP_HIP(hipMemsetAsync(flags, 0, 4, stream));
    if (nnz > 0) {
        hipLaunchKernelGGL(k_check_entries, dim3(grid_for(nnz)), dim3(kBlock), 0, stream, lp.a_col, lp.a_val, nnz,
                           lp.n, flags);
        hipLaunchKernelGGL(k_check_entries, dim3(grid_for(nnz)), dim3(kBlock), 0, stream, lp.at_col, lp.at_val,
                           nnz, lp.m, flags);
    }
    hipLaunchKernelGGL(k_check_vec, dim3(grid_for(lp.m)), dim3(kBlock), 0, stream, lp.b, (int64_t)lp.m, flags);
    hipLaunchKernelGGL(k_check_vec, dim3(grid_for(lp.n)), dim3(kBlock), 0, stream, lp.c, (int64_t)lp.n, flags);
    if (has_bounds(lp))
        hipLaunchKernelGGL(k_check_bounds, dim3(grid_for(lp.n)), dim3(kBlock), 0, stream, lp.lo, lp.hi,
                           (int64_t)lp.n, flags);
    if (has_sense(lp))
        hipLaunchKernelGGL(k_check_sense, dim3(grid_for(lp.m)), dim3(kBlock), 0, stream, lp.sense, (int64_t)lp.m,
                           flags);
    MIP_LAUNCH_CHECK();
    int32_t f = 0;
    MIP_HIP(hipMemcpyAsync(&f, flags, 4, hipMemcpyDeviceToHost, stream));
    MIP_HIP(hipStreamSynchronize(stream));
    if (f & 1) return set_error("column index out of range"), MIPDHG_ERR_BAD_CSR;
    if (f & 6) return set_error("NaN or Inf in A, A^T, b or c"), MIPDHG_ERR_NONFINITE;
    if (f & 8) return set_error("a bound is NaN, lo = +inf, hi = -inf or lo > hi"), MIPDHG_ERR_INVALID_ARG;
    if (f & 16) return set_error("a row sense is not 0, 1 or 2"), MIPDHG_ERR_INVALID_ARG;
    if (nnz == 0) return 0;
    // u^T (A v) against v^T (A^T u), and the scale sum |u||A||v|
    const uint32_t su = 0x1234u, sv = 0xABCDu;
    hipLaunchKernelGGL((k_transpose_dot<false>), dim3(ta.ntiles), dim3(kBlock), tile_lds_bytes(ta, 8), stream, ta, lp.a_col,
                       lp.a_val, su, sv, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, stream, (const double*)partials, ta.ntiles, red);
    hipLaunchKernelGGL((k_transpose_dot<true>), dim3(ta.ntiles), dim3(kBlock), tile_lds_bytes(ta, 8), stream, ta, lp.a_col,
                       lp.a_val, su, sv, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, stream, (const double*)partials, ta.ntiles,
                       red + 1);
    hipLaunchKernelGGL((k_transpose_dot<false>), dim3(tat.ntiles), dim3(kBlock), tile_lds_bytes(tat, 8), stream, tat, lp.at_col,
                       lp.at_val, sv, su, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, stream, (const double*)partials, tat.ntiles,
                       red + 2);
    hipLaunchKernelGGL((k_transpose_dot<true>), dim3(tat.ntiles), dim3(kBlock), tile_lds_bytes(tat, 8), stream, tat, lp.at_col,
                       lp.at_val, sv, su, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, stream, (const double*)partials, tat.ntiles,
                       red + 3);
    MIP_LAUNCH_CHECK();
    double r[4];
    MIP_HIP(hipMemcpyAsync(r, red, 4 * 8, hipMemcpyDeviceToHost, stream));
    MIP_HIP(hipStreamSynchronize(stream));
    const double scale = std::max(r[1], r[3]);
    if (!(fabs(r[0] - r[2]) <= 1e-10 * scale + 1e-300))
        return set_error("A^T does not match A (dot test %.17g vs %.17g)", r[0], r[2]), MIPDHG_ERR_TRANSPOSE;
    return 0;
}

}  // namespace mip
