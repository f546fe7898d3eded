// Shared device helpers and host plumbing for the mipdhg HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <vector>

#include "mipdhg.h"

namespace mip {

constexpr int kBlock = 256;  // threads per workgroup for the row kernels (4 waves)
constexpr int kWave = 64;    // CDNA wavefront
constexpr int kMaxShortBlocks = 2048;  // 8 resident workgroups x 256 CUs
constexpr int kMaxLongBlocks = 1024;
constexpr int kMaxRowBlocks = kMaxShortBlocks + kMaxLongBlocks;

// ---------------------------------------------------------------------------
// host error plumbing
// ---------------------------------------------------------------------------
void set_error(const char* fmt, ...);
void clear_error();

#define MIP_HIP(expr)                                                              \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            ::mip::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                             __FILE__, __LINE__);                                  \
            return MIPDHG_ERR_HIP;                                                 \
        }                                                                          \
    } while (0)

#define MIP_LAUNCH_CHECK()                                                          \
    do {                                                                            \
        hipError_t e_ = hipGetLastError();                                          \
        if (e_ != hipSuccess) {                                                     \
            ::mip::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), \
                             __FILE__, __LINE__);                                   \
            return MIPDHG_ERR_HIP;                                                  \
        }                                                                           \
    } while (0)

// ---------------------------------------------------------------------------
// loads
// ---------------------------------------------------------------------------
// Matrix values and column indices are streamed once per SpMV: non-temporal
// loads keep them from evicting the gathered vector from L2.
__device__ __forceinline__ double ld_val(const double* p, int64_t k) {
    return __builtin_nontemporal_load(p + k);
}
__device__ __forceinline__ float ld_val(const float* p, int64_t k) {
    return __builtin_nontemporal_load(p + k);
}
// bfloat16 stored as its upper 16 bits
__device__ __forceinline__ float ld_val(const uint16_t* p, int64_t k) {
    uint32_t b = __builtin_nontemporal_load(p + k);
    return __uint_as_float(b << 16);
}
__device__ __forceinline__ int32_t ld_idx(const int32_t* p, int64_t k) {
    return __builtin_nontemporal_load(p + k);
}
// Cached loads of values re-read every iteration by the same workgroup (a
// batched instance's matrix stays in L2 between its iterations).
__device__ __forceinline__ double ld_val_cached(const double* p, int64_t k) { return p[k]; }
__device__ __forceinline__ float ld_val_cached(const float* p, int64_t k) { return p[k]; }
__device__ __forceinline__ float ld_val_cached(const uint16_t* p, int64_t k) {
    return __uint_as_float((uint32_t)p[k] << 16);
}

// Element i of an array whose base the whole wavefront shares, addressed as
// that base plus a 32-bit byte offset (the offset must stay below 4 GiB):
// one vector register per address instead of two.
template <typename T>
__device__ __forceinline__ const T* at(const T* base, uint32_t i) {
    return (const T*)((const char*)base + (uint64_t)(i * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ T* at(T* base, uint32_t i) {
    return (T*)((char*)base + (uint64_t)(i * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ T ld_at(const T* base, uint32_t i) {
    return *at(base, i);
}
template <typename T>
__device__ __forceinline__ T ld_at_nt(const T* base, uint32_t i) {
    return __builtin_nontemporal_load(at(base, i));
}
template <typename T>
__device__ __forceinline__ void st_at(T* base, uint32_t i, T v) {
    *at(base, i) = v;
}
__device__ __forceinline__ double ld_val_at(const double* p, uint32_t i) { return ld_at_nt(p, i); }
__device__ __forceinline__ float ld_val_at(const float* p, uint32_t i) { return ld_at_nt(p, i); }
__device__ __forceinline__ float ld_val_at(const uint16_t* p, uint32_t i) {
    const uint32_t b = ld_at_nt(p, i);
    return __uint_as_float(b << 16);
}

// float -> bfloat16 with round-to-nearest-even (finite inputs)
__host__ __device__ inline uint16_t f32_to_bf16_rne(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

template <typename V> struct ValueOf;
template <> struct ValueOf<double> { typedef double acc; };
template <> struct ValueOf<float> { typedef float acc; };
template <> struct ValueOf<uint16_t> { typedef float acc; };

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
template <int L, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, L);
    return v;
}

template <typename T>
__device__ __forceinline__ T group_sum_rt(T v, int L) {
    for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, L);
    return v;
}

template <typename T>
__device__ __forceinline__ T group_max_rt(T v, int L) {
    for (int o = L / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, L));
    return v;
}

// Block-wide reduction of NS sums and NM maxima, in a fixed order, written to
// out[q] for q in [0, NS+NM) whose bit is set in `mask`.  Every thread of the
// block must call it.
template <int NS, int NM, int BS = kBlock>
__device__ __forceinline__ void block_reduce_store(double (&s)[NS], double (&mx)[NM > 0 ? NM : 1],
                                                   double* out, unsigned mask = ~0u) {
    __shared__ double sh[(NS + NM) > 0 ? (NS + NM) : 1][BS / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        double v = group_sum<kWave>(s[q]);
        if (lane == 0) sh[q][wave] = v;
    }
#pragma unroll
    for (int q = 0; q < NM; ++q) {
        double v = mx[q];
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
        if (lane == 0) sh[NS + q][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < NS + NM) {
        const int q = threadIdx.x;
        double v = sh[q][0];
        for (int w = 1; w < BS / kWave; ++w) v = (q < NS) ? v + sh[q][w] : fmax(v, sh[q][w]);
        if (mask & (1u << q)) out[q] = v;
    }
}

// ---------------------------------------------------------------------------
// row plans: which workgroup handles which CSR rows
// ---------------------------------------------------------------------------
// Rows no longer than `long_thresh` are handled by groups of `lanes` lanes;
// each of the first g_short workgroups owns a contiguous chunk of rows.
// Longer rows (listed in long_rows) are handled one wavefront per row by the
// g_long workgroups after them.  Workgroups are dispatched round-robin over
// the 8 XCDs; xcd_virtual_block() gives each XCD a contiguous run of chunks so
// that the vector entries a chunk gathers stay in that XCD's L2.
struct RowPlan {
    const int32_t* rowptr;
    const int32_t* long_rows;
    int32_t nrows;
    int32_t nlong;
    int32_t long_thresh;
    int32_t lanes;
    int32_t chunk;
    int32_t g_short;
    int32_t g_long;
    int32_t pad;
};

__device__ __forceinline__ int xcd_virtual_block(int b, int G) {
    const int q = G >> 3, r = G & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

// The tile of a launch with one workgroup per tile.
__device__ __forceinline__ int own_tile() { return xcd_virtual_block(blockIdx.x, gridDim.x); }

// The tiles of a persistent launch: the descriptors form 8 contiguous runs,
// one per XCD (workgroups b and b + 8 run on the same XCD), and the workgroups of an XCD
// stride over its run.  Covers [0, ntiles) exactly once for any grid that
// has at least min(8, ntiles) workgroups.
struct TileRange {
    int first, end, step;
};
__device__ __forceinline__ TileRange persistent_tiles(int ntiles) {
    const int G = gridDim.x, b = blockIdx.x, x = b & 7;
    const int q = ntiles >> 3, r = ntiles & 7;
    const int t0 = x * q + min(x, r);
    return TileRange{t0 + (b >> 3), t0 + q + (x < r ? 1 : 0), (G >> 3) + (x < (G & 7) ? 1 : 0)};
}

// Visit every row of the plan.  dot(s, e, lane, L) returns this lane's share of
// the row's reduction; epi(row, total) runs on the group's first lane.
template <int L, typename Acc, class Dot, class Epi>
__device__ __forceinline__ void for_rows(const RowPlan& p, Dot dot, Epi epi) {
    const int b = blockIdx.x;
    if (b < p.g_short) {
        const int vb = xcd_virtual_block(b, p.g_short);
        const int r0 = vb * p.chunk;
        const int r1 = min(r0 + p.chunk, p.nrows);
        constexpr int GPB = kBlock / L;
        const int grp = threadIdx.x / L;
        const int lane = threadIdx.x & (L - 1);
        for (int r = r0 + grp; r < r1; r += GPB) {
            const int s = p.rowptr[r];
            const int e = p.rowptr[r + 1];
            if (e - s > p.long_thresh) continue;
            Acc acc = dot(s, e, lane, L);
            acc = group_sum<L>(acc);
            if (lane == 0) epi(r, acc);
        }
    } else {
        const int lb = b - p.g_short;
        const int wave = threadIdx.x / kWave;
        const int lane = threadIdx.x & (kWave - 1);
        for (int li = lb * (kBlock / kWave) + wave; li < p.nlong; li += p.g_long * (kBlock / kWave)) {
            const int r = p.long_rows[li];
            const int s = p.rowptr[r];
            const int e = p.rowptr[r + 1];
            Acc acc = dot(s, e, lane, kWave);
            acc = group_sum<kWave>(acc);
            if (lane == 0) epi(r, acc);
        }
    }
}

// ---------------------------------------------------------------------------
// nnz-balanced tiles staged through LDS
// ---------------------------------------------------------------------------
// A tile is a run of consecutive rows holding at most tile_nnz nonzeros and
// tile_rows rows; a row with more than tile_nnz nonzeros is a tile of its own
// ("huge" row).  One workgroup per tile:
//   0. the epilogue's per-row vector reads for the tile's rows are issued
//      (Epi::load) so that their latency overlaps the products;
//   1. the tile's row offsets go to LDS and every product val[k]*x[col[k]] of
//      the tile is computed with tile_nnz/kBlock independent gathers per
//      thread and stored in LDS;
//   2. rows of at most short_row products are summed by one thread each, the
//      longer rows (listed in row order) by one wavefront each; sums go to LDS;
//   3. the epilogue runs for all rows in parallel, one thread per row, so its
//      vector reads and writes are coalesced.
// Every sum is taken in a fixed order, so results do not depend on timing.
// `active` (uniform) is checked after the products, before anything is
// written: a kernel can load its control word early and still be a no-op.
constexpr int kTileNnzDefault = 2048;
constexpr int kTileRowsDefault = 512;
constexpr int kShortRowDefault = -1;  // chunked segmented row sums
constexpr int kMaxTileRows = 512;   // bound of the per-thread prefetch
constexpr int kMaxTileNnz = 8192;
constexpr int kRowsPerThread = kMaxTileRows / kBlock;

struct TilePlan {
    const int32_t* rowptr;
    const int4* desc;  // [ntiles] {first row, end row, first nonzero, end nonzero},
                       // in the order the workgroups take them (see make_tile_desc)
    int32_t ntiles;
    int32_t nrows;
    int32_t tile_nnz;   // nonzeros per tile (LDS products)
    int32_t tile_rows;  // rows per tile, <= kMaxTileRows
    int32_t short_row;  // rows up to this length are summed by one thread
    int32_t max_long;   // tile_nnz / (short_row + 1) + 1
    // Sorted layout: nonzero k of a tile (other than a one-row tile) holds the
    // product whose row-major position in the tile is slot[k]; nullptr for
    // the row-major layout.
    const uint16_t* slot;
};

// Product slots of a tile: tile_nnz rounded up to a whole number of the
// largest chunk (32), so that rotated chunks stay inside; one more slot
// after them is a dummy target for out-of-range lanes.
__host__ __device__ inline int prod_cap(const TilePlan& p) { return (p.tile_nnz + 31) & ~31; }

// The tile's LDS, carved from dynamic shared memory.
template <typename Acc>
struct TileLds {
    Acc* prod;
    Acc* sum;
    Acc* wsum;  // per-wave scan totals of the chunked reduction
    int32_t* row;
    int32_t* list;
    int32_t* wcount;
};

template <typename Acc>
__device__ __forceinline__ TileLds<Acc> tile_lds(unsigned char* smem, const TilePlan& p) {
    TileLds<Acc> L;
    L.prod = (Acc*)smem;
    L.sum = L.prod + prod_cap(p) + 1;  // prod[prod_cap] is a dummy slot
    L.wsum = L.sum + p.tile_rows;
    L.row = (int32_t*)(L.wsum + kBlock / kWave);
    L.list = L.row + p.tile_rows + 1;
    L.wcount = L.list + p.max_long;
    return L;
}

inline size_t tile_lds_bytes(const TilePlan& p, size_t acc) {
    return acc * (size_t)(prod_cap(p) + 1 + p.tile_rows + kBlock / kWave) +
           4 * (size_t)(p.tile_rows + 1 + p.max_long + kBlock / kWave) + 16;
}

template <bool MAXOP, typename Acc>
__device__ __forceinline__ Acc red_op(Acc a, Acc b) {
    return MAXOP ? (a > b ? a : b) : a + b;
}

template <bool MAXOP, typename Acc>
__device__ __forceinline__ Acc wave_red(Acc v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = red_op<MAXOP>(v, __shfl_xor(v, o, kWave));
    return v;
}

// Epilogue without prefetched values, from a lambda f(row, sum).
struct NoPre {};
template <class F>
struct LambdaEpi {
    F f;
    typedef NoPre Pre;
    __device__ __forceinline__ void ready() {}
    __device__ __forceinline__ bool running() const { return true; }
    __device__ __forceinline__ NoPre load(int, int) const { return NoPre{}; }
    template <class A>
    __device__ __forceinline__ void apply(int r0, int i, const NoPre&, A s) const {
        f(r0 + i, s);
    }
};
template <class F>
__device__ __forceinline__ LambdaEpi<F> lepi(F f) {
    return LambdaEpi<F>{f};
}

// Row totals of a tile whose products are in L.prod and whose row offsets
// (relative to the tile) are in L.row[0..nr].  Every thread reduces one
// contiguous chunk of C = 2^lgc >= nz / 256 products, stored swizzled inside
// the chunk (chunk_slot) so that the lanes, which read their chunks in step,
// fall on different LDS banks.  Rows that end inside the chunk
// after its first row end are complete and written at once; the part of the
// first row that ends in the chunk needs what earlier threads hold of that
// row, which a segmented scan over the threads supplies (a chunk with a row
// end starts a new segment of the scan).  Empty rows keep the 0 written to
// L.sum beforehand.  The work per thread does not depend on the row lengths.
// log2 of the chunk length for nz products over the 256 threads
__device__ __forceinline__ int chunk_lg(int nz) {
    const int c = (nz + kBlock - 1) / kBlock;
    return c <= 1 ? 0 : 32 - __clz(c - 1);
}

// LDS position of product k: inside its chunk of 2^lgc products the
// position is XORed with bits of the chunk number, so that the lanes of a
// wavefront, which read their chunks in step, are spread evenly over the LDS
// banks (the chunk of thread t starts at double 2^lgc t; lanes whose chunks
// start on the same bank get different XOR values).  Identity for lgc = 0.
__device__ __forceinline__ int chunk_slot(int k, int lgc) {
    return k ^ ((k >> 5) & ((1 << lgc) - 1));
}

template <bool MAXOP, typename Acc>
__device__ __forceinline__ void chunk_row_sums(const TileLds<Acc>& L, int nz, int nr, int lgc) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int C = 1 << lgc;
    const int p0 = tid * C, p1 = min(p0 + C, nz);
    const Acc* mine = L.prod + p0;  // product k at mine[(k - p0) ^ x]
    const int x = (p0 >> 5) & (C - 1);
    bool ends = false;  // a row ends inside this chunk
    Acc head = 0, acc = 0;
    int rfirst = 0;
    if (p0 < nz) {
        int lo = 0, hi = nr;  // row[lo] <= p0 < row[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (L.row[mid] <= p0) lo = mid;
            else hi = mid;
        }
        int r = lo, end = L.row[lo + 1];
        rfirst = r;
        for (int k = p0; k < p1; ++k) {
            acc = red_op<MAXOP>(acc, mine[(k - p0) ^ x]);
            if (k + 1 == end) {
                if (ends) L.sum[r] = acc;
                else head = acc;
                ends = true;
                acc = 0;
                do {  // next non-empty row
                    ++r;
                    end = r < nr ? L.row[r + 1] : 0x7fffffff;
                } while (end == k + 1);
            }
        }
    }
    // inclusive segmented scan of (ends, open tail) over the wave; the
    // earlier operand is always on the left
    Acc v = acc;
    int f = ends ? 1 : 0;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const Acc v2 = __shfl_up(v, d, kWave);
        const int f2 = __shfl_up(f, d, kWave);
        if (lane >= d) {
            if (!f) v = red_op<MAXOP>(v2, v);
            f |= f2;
        }
    }
    if (lane == kWave - 1) {
        L.wsum[wave] = v;
        L.wcount[wave] = f;
    }
    Acc ev = __shfl_up(v, 1, kWave);
    int ef = __shfl_up(f, 1, kWave);
    if (lane == 0) {
        ev = 0;
        ef = 0;
    }
    __syncthreads();
    Acc pv = 0;  // the waves before this one
    for (int w = 0; w < wave; ++w) pv = L.wcount[w] ? L.wsum[w] : red_op<MAXOP>(pv, L.wsum[w]);
    const Acc carry = ef ? ev : red_op<MAXOP>(pv, ev);
    if (ends) L.sum[rfirst] = red_op<MAXOP>(carry, head);
}

// prod(b, j) -> Acc for nonzero b + j, with b the same in the whole
// workgroup and 0 <= j < 65536.  Epi provides Pre load(r0, i) and
// apply(r0, i, pre, total) for row r0 + i of a tile starting at row r0.
template <bool MAXOP, typename Acc, int U = 8, bool SORTED = false, class Prod, class Epi>
__device__ __forceinline__ void tiled_rows(const TilePlan& p, int tile, const TileLds<Acc>& L, Prod prod,
                                           Epi& epi, bool active = true) {
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const int4 d = p.desc[tile];
    const int r0 = d.x, r1 = d.y, s = d.z, e = d.w;
    const int nr = r1 - r0;
    const int nz = e - s;
    if (nz > p.tile_nnz) {  // one huge row: the whole workgroup strides over it
        typename Epi::Pre pre0;
        if (tid == 0) pre0 = epi.load(r0, 0);
        Acc a = 0;
        for (int k0 = s; k0 < e; k0 += kBlock)
            if (k0 + tid < e) a = red_op<MAXOP>(a, prod(k0, tid));
        a = wave_red<MAXOP>(a);
        if (lane == 0) L.prod[wave] = a;
        epi.ready();
        __syncthreads();
        if (tid == 0 && active && epi.running()) {
            Acc tot = L.prod[0];
            for (int w = 1; w < kBlock / kWave; ++w) tot = red_op<MAXOP>(tot, L.prod[w]);
            epi.apply(r0, 0, pre0, tot);
        }
        return;
    }
    // Every load that does not depend on another is issued here, branch-free
    // (indices clamped into the tile), so that their latencies overlap: the
    // epilogue's vector entries, the row offsets, and the matrix entries of
    // the first products.
    typename Epi::Pre pre[kRowsPerThread];
#pragma unroll
    for (int q = 0; q < kRowsPerThread; ++q) pre[q] = epi.load(r0, min(tid + q * kBlock, nr - 1));
    int rp[kRowsPerThread + 1];
#pragma unroll
    for (int q = 0; q <= kRowsPerThread; ++q) rp[q] = ld_at(p.rowptr + r0, min(tid + q * kBlock, nr));
    // products, U per thread in flight
    const bool chunked = p.short_row < 0;
    const int lgc = chunked ? chunk_lg(nz) : 0;  // 0: no rotation
    for (int base = 0; base < nz; base += U * kBlock) {
        Acc v[U];
        int sl[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = min(base + tid + u * kBlock, nz - 1);
            v[u] = prod(s, j);
            sl[u] = SORTED ? (int)ld_at_nt(p.slot + s, j) : j;
        }
        // out-of-range lanes store to the dummy slot prod[prod_cap], so the
        // stores need no branch
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = base + tid + u * kBlock;
            L.prod[k < nz ? chunk_slot(sl[u], lgc) : prod_cap(p)] = v[u];
        }
    }
#pragma unroll
    for (int q = 0; q <= kRowsPerThread; ++q)
        if (tid + q * kBlock <= nr) L.row[tid + q * kBlock] = rp[q] - s;
    epi.ready();
    if (chunked)
#pragma unroll
        for (int q = 0; q < kRowsPerThread; ++q)
            if (tid + q * kBlock < nr) L.sum[tid + q * kBlock] = 0;
    __syncthreads();
    if (!active || !epi.running()) return;  // uniform
    if (chunked) {
        chunk_row_sums<MAXOP>(L, nz, nr, lgc);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kRowsPerThread; ++q) {
            const int i = tid + q * kBlock;
            if (i < nr) epi.apply(r0, i, pre[q], L.sum[i]);
        }
        return;
    }
    int nlist = 0;
    for (int base = 0; base < nr; base += kBlock) {
        const int i = base + tid;
        bool lng = false;
        if (i < nr) {
            const int a = L.row[i], b = L.row[i + 1];
            if (b - a <= p.short_row) {
                // each lane starts at its own offset inside the row and wraps
                // around: row starts that differ by a multiple of the bank
                // count would otherwise hit one LDS bank on every step
                const int len = b - a;
                const int j0 = len > 0 ? (lane & ((1 << (31 - __clz(len))) - 1)) : 0;
                Acc acc = 0;
                int q = a + j0;
                for (int c = 0; c < len; ++c) {
                    acc = red_op<MAXOP>(acc, L.prod[q]);
                    q = (q + 1 == b) ? a : q + 1;
                }
                L.sum[i] = acc;
            } else {
                lng = true;
            }
        }
        // rows too long for one thread, appended to the list in row order
        const unsigned long long mask = __ballot(lng);
        if (lane == 0) L.wcount[wave] = __popcll(mask);
        __syncthreads();
        int off = nlist;
        for (int w = 0; w < wave; ++w) off += L.wcount[w];
        int tot = 0;
        for (int w = 0; w < kBlock / kWave; ++w) tot += L.wcount[w];
        if (lng) L.list[off + __popcll(mask & ((1ull << lane) - 1ull))] = i;
        nlist += tot;
        __syncthreads();
    }
    for (int j = wave; j < nlist; j += kBlock / kWave) {
        const int i = L.list[j];
        const int a = L.row[i], b = L.row[i + 1];
        Acc acc = 0;
        for (int q = a + lane; q < b; q += kWave) acc = red_op<MAXOP>(acc, L.prod[q]);
        acc = wave_red<MAXOP>(acc);
        if (lane == 0) L.sum[i] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kRowsPerThread; ++q) {
        const int i = tid + q * kBlock;
        if (i < nr) epi.apply(r0, i, pre[q], L.sum[i]);
    }
}

// Tiles of the rows, as 4 ints per tile in workgroup order (see plain.hip).
std::vector<int32_t> make_tile_desc(const std::vector<int32_t>& rowptr, int32_t nrows, int32_t tile_nnz,
                                    int32_t tile_rows);
bool tile_desc_ok(const std::vector<int32_t>& desc, const std::vector<int32_t>& rowptr, int32_t nrows,
                  int32_t tile_nnz, int32_t tile_rows);
inline int64_t max_tiles(int64_t nrows, int64_t nnz, int64_t tile_nnz, int64_t tile_rows) {
    return 2 * (nnz / tile_nnz + nrows / tile_rows) + 4;
}

// Run-time lane count dispatch for the setup kernels.
#define MIP_DISPATCH_L(LANES, ...)                        \
    switch (LANES) {                                      \
        case 2: { constexpr int L = 2; __VA_ARGS__; } break;   \
        case 4: { constexpr int L = 4; __VA_ARGS__; } break;   \
        case 8: { constexpr int L = 8; __VA_ARGS__; } break;   \
        case 16: { constexpr int L = 16; __VA_ARGS__; } break; \
        case 32: { constexpr int L = 32; __VA_ARGS__; } break; \
        default: { constexpr int L = 64; __VA_ARGS__; } break; \
    }

// Host-side plan: lane count and long-row list from the row pointers.
struct HostPlan {
    int32_t lanes = 8;
    int32_t long_thresh = 128;
    int32_t chunk = 0;
    int32_t g_short = 0;
    int32_t g_long = 0;
    std::vector<int32_t> long_rows;
    int32_t grid() const { return g_short + g_long; }
};

HostPlan make_plan(const std::vector<int32_t>& rowptr, int32_t nrows, int32_t lanes_opt,
                   int32_t long_opt);
RowPlan device_plan(const HostPlan& hp, const int32_t* rowptr, const int32_t* long_rows_dev,
                    int32_t nrows);

// workspace carving
struct Carver {
    char* base;
    size_t off = 0;
    size_t cap;
    explicit Carver(void* b, size_t c) : base((char*)b), cap(c) {}
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

}  // namespace mip
