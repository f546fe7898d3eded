// Centered start point of Algorithm 1 (Section 3.1): the map from a PDHG
// solution of the scaled LP to the interior-point warm start, and the
// alpha_min re-clamp of its step-recovery loop.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "common.h"
#include "plain.h"

namespace mip {

// Optionally scales an original-space (x, z) to the scaled LP
// (x~ = x / d_col, z~ = z * d_col), kept in xs/zs unless they are NULL;
// partial sums of x~_j z~_j.
__global__ __launch_bounds__(kBlock) void k_center_dot(const double* x, const double* z, const double* d_col,
                                                       int64_t n, double* xs, double* zs, double* partials) {
    double s[1] = {0.0};
    double mx[1] = {0.0};
    for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
        double xv = x[j], zv = z[j];
        if (d_col) {
            xv = xv / d_col[j];
            zv = zv * d_col[j];
        }
        if (xs) {
            xs[j] = xv;
            zs[j] = zv;
        }
        s[0] += xv * zv;
    }
    block_reduce_store<1, 0>(s, mx, partials + blockIdx.x);
}

// mu_target = max(sum(partials) / n, mu_min), fixed-order sum in one workgroup
__global__ __launch_bounds__(kBlock) void k_center_mu(const double* partials, int G, int64_t n, double mu_min,
                                                      double* mu) {
    __shared__ double sh[kBlock];
    double s = 0.0;
    for (int g = threadIdx.x; g < G; g += kBlock) s += partials[g];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *mu = fmax(sh[0] / (double)n, mu_min);
}

// v moved to target, but by at most delta
__device__ __forceinline__ double pull(double v, double target, double delta) {
    return fmin(fmax(target, v - delta), v + delta);
}

// The centring map of one pair, both members raised to alpha first: the
// strictly smaller member (z on a tie) is pulled toward mu / (the other),
// then the other toward mu / (the first's new value), each by at most delta.
__device__ __forceinline__ void center_pair(double xv, double zv, double mu, double delta, double alpha,
                                            double& xo, double& zo) {
    const double xl = fmax(xv, alpha), zl = fmax(zv, alpha);
    const bool x_first = xl < zl;
    double first = x_first ? xl : zl, second = x_first ? zl : xl;
    first = pull(first, mu / second, delta);
    second = pull(second, mu / first, delta);
    xo = x_first ? first : second;
    zo = x_first ? second : first;
}

// the map over all pairs of an already scaled (xs, zs)
__global__ void k_center_map(const double* xs, const double* zs, int64_t n, const double* mu_p, double delta,
                             double alpha, double* xo, double* zo) {
    const double mu = *mu_p;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        center_pair(xs[j], zs[j], mu, delta, alpha, xo[j], zo[j]);
}

__global__ void k_reclamp(double* x, double* z, int64_t n, double alpha) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        x[j] = fmax(x[j], alpha);
        z[j] = fmax(z[j], alpha);
    }
}

}  // namespace mip

using namespace mip;

namespace {

// Bytes the centring needs for n pairs: the partial sums of x~ z~ (one per
// workgroup, at most 1,024), the target mu, and the scaled copies x~, z~.
constexpr size_t center_bytes(int64_t n) {
    const int64_t g = (n + kBlock - 1) / kBlock;
    const int64_t G = g < 1 ? 1 : (g > 1024 ? 1024 : g);
    return ((size_t)G * 8 + 255) / 256 * 256 + 256 + 2 * (((size_t)n * 8 + 255) / 256 * 256);
}

// The allocation-free entry point keeps its scratch in this array: every
// GPU the library runs on holds its own copy (33.6 MB) until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is a stand-in, not a device address); it uses the address that
// hipGetSymbolAddress returns for the current device.
constexpr int32_t kNoAllocMaxN = 1 << 21;
constexpr size_t kNoAllocBytes = center_bytes(kNoAllocMaxN);

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's scratch array, looked up once
// per device (with that device current) and kept.
int scratch_of_current_device(void** out) {
    int dev = -1;
    MIP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error("device ordinal %d out of range", dev), MIPDHG_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error("hipGetSymbolAddress of the centring scratch failed: %s", hipGetErrorString(e)),
                   MIPDHG_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

int check_center_args(int32_t n, const double* x, const double* z, double mu_min, double delta_max,
                      double alpha_min, const double* x_out, const double* z_out) {
    if (n < 1 || !x || !z || !x_out || !z_out)
        return set_error("n >= 1 and non-NULL x, z, x_out, z_out are required"), MIPDHG_ERR_INVALID_ARG;
    if (!(mu_min > 0.0) || !(delta_max >= 0.0) || !(alpha_min >= 0.0) || !std::isfinite(mu_min) ||
        !std::isfinite(delta_max) || !std::isfinite(alpha_min))
        return set_error("need mu_min > 0, delta_max >= 0, alpha_min >= 0, all finite"), MIPDHG_ERR_INVALID_ARG;
    return 0;
}

// The three launches of the centring on a buffer of center_bytes(n) bytes.
int center_run(int32_t n, const double* x, const double* z, const double* d_col, double mu_min, double delta_max,
               double alpha_min, void* buf, size_t bytes, hipStream_t s, double* x_out, double* z_out,
               double* mu_target) {
    Carver cv(buf, bytes);
    const int G = grid_for(n, 1024);
    double* partials = cv.take<double>(G);
    double* mu = cv.take<double>(32);
    double* xs = cv.take<double>(n);
    double* zs = cv.take<double>(n);
    hipLaunchKernelGGL(k_center_dot, dim3(G), dim3(kBlock), 0, s, x, z, d_col, (int64_t)n, xs, zs, partials);
    hipLaunchKernelGGL(k_center_mu, dim3(1), dim3(kBlock), 0, s, (const double*)partials, G, (int64_t)n, mu_min, mu);
    hipLaunchKernelGGL(k_center_map, dim3(grid_for(n)), dim3(kBlock), 0, s, (const double*)xs, (const double*)zs,
                       (int64_t)n, (const double*)mu, delta_max, alpha_min, x_out, z_out);
    MIP_LAUNCH_CHECK();
    if (mu_target) MIP_HIP(hipMemcpyAsync(mu_target, mu, 8, hipMemcpyDeviceToHost, s));
    MIP_HIP(hipStreamSynchronize(s));
    return 0;
}

}  // namespace

extern "C" size_t mipdhg_center_workspace_size(int32_t n) { return center_bytes(n); }

extern "C" int mipdhg_center_start(int32_t n, const double* x, const double* z, const double* d_col, double mu_min,
                                   double delta_max, double alpha_min, void* workspace, size_t workspace_bytes,
                                   void* stream, double* x_out, double* z_out, double* mu_target) {
    clear_error();
    int rc = check_center_args(n, x, z, mu_min, delta_max, alpha_min, x_out, z_out);
    if (rc) return rc;
    if (!workspace) return set_error("workspace is NULL"), MIPDHG_ERR_INVALID_ARG;
    if (workspace_bytes < mipdhg_center_workspace_size(n))
        return set_error("workspace too small"), MIPDHG_ERR_WORKSPACE;
    if (((uintptr_t)workspace & 255) != 0) return set_error("workspace must be 256-byte aligned"), MIPDHG_ERR_INVALID_ARG;
    return center_run(n, x, z, d_col, mu_min, delta_max, alpha_min, workspace, workspace_bytes, (hipStream_t)stream,
                      x_out, z_out, mu_target);
}

extern "C" int32_t mipdhg_center_noalloc_max_n(void) { return kNoAllocMaxN; }

extern "C" int mipdhg_center_start_noalloc(int32_t n, const double* x, const double* z, const double* d_col,
                                           double mu_min, double delta_max, double alpha_min, void* stream,
                                           double* x_out, double* z_out, double* mu_target) {
    clear_error();
    int rc = check_center_args(n, x, z, mu_min, delta_max, alpha_min, x_out, z_out);
    if (rc) return rc;
    if (n > kNoAllocMaxN)
        return set_error("n = %d is more than the %d pairs the allocation-free scratch holds; "
                         "use mipdhg_center_start with a workspace", n, kNoAllocMaxN),
               MIPDHG_ERR_INVALID_ARG;
    void* buf = nullptr;
    if ((rc = scratch_of_current_device(&buf))) return rc;
    return center_run(n, x, z, d_col, mu_min, delta_max, alpha_min, buf, kNoAllocBytes, (hipStream_t)stream, x_out,
                      z_out, mu_target);
}

extern "C" int mipdhg_center_reclamp(int32_t n, double alpha_min, void* stream, double* x_io, double* z_io) {
    clear_error();
    if (n < 1 || !x_io || !z_io || !(alpha_min >= 0.0) || !std::isfinite(alpha_min))
        return set_error("n >= 1, non-NULL vectors and a finite alpha_min >= 0 are required"), MIPDHG_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_reclamp, dim3(grid_for(n)), dim3(kBlock), 0, s, x_io, z_io, (int64_t)n, alpha_min);
    MIP_LAUNCH_CHECK();
    MIP_HIP(hipStreamSynchronize(s));
    return 0;
}

