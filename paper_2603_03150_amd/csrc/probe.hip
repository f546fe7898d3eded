// Streaming-read probe: a plain read of a device buffer of known size, the
// same non-temporal 16-byte vector loads the SpMV kernels stream their
// matrices with.  Timing it gives the read rate a kernel can reach on the
// device; profiling it gives the bytes a hardware read counter reports for a
// known number of bytes read.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"
#include "mipdhg.h"

using namespace mip;

namespace {

typedef unsigned pu4 __attribute__((ext_vector_type(4)));
constexpr int kProbeBlock = 256;
constexpr int kProbeUnroll = 4;

// Every 16-byte word is read once: thread t of the grid takes words
// t + k * stride, kProbeUnroll of them per step with all loads in flight
// together.  The words are folded with XOR so that the loads are kept; one
// word per wave is written.
__global__ __launch_bounds__(kProbeBlock) void k_read_probe(const pu4* __restrict__ p, int64_t n16,
                                                              unsigned* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * kProbeBlock;
    unsigned acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x; i < n16; i += kProbeUnroll * stride) {
        pu4 v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const int64_t j = i + u * stride;
            v[u] = j < n16 ? __builtin_nontemporal_load(p + j) : pu4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) acc ^= __shfl_xor(acc, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) out[((int64_t)blockIdx.x * kProbeBlock + threadIdx.x) / kWave] = acc;
}

}  // namespace

extern "C" int mipdhg_read_probe(const void* buf, size_t bytes, int32_t blocks, void* stream, uint32_t* out) {
    clear_error();
    if (!buf || !out || bytes == 0 || bytes % 16 != 0 || ((uintptr_t)buf & 15) != 0 || blocks < 1)
        return set_error("a 16-byte aligned buffer, a size that is a positive multiple of 16, blocks >= 1 and an "
                         "output are required"),
               MIPDHG_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_read_probe, dim3(blocks), dim3(kProbeBlock), 0, (hipStream_t)stream, (const pu4*)buf,
                       (int64_t)(bytes / 16), (unsigned*)out);
    MIP_LAUNCH_CHECK();
    return 0;
}
