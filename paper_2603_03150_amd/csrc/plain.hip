// Restarted PDHG for one standard-form LP: kernels and host driver.
//
// The iteration runs on the scaled problem (Section 2.1 asks for scaling; the
// scheme is Ruiz + Pock-Chambolle).  Every `eval_every` iterations the
// projected point is unscaled and measured on the caller's float64 A, and the
// three relative tests of Section 2 decide termination; restarts and the primal
// weight follow the cuPDLP+ family that Section 4.1 names.
//
// Per iteration two fused kernels run:
//   primal (rows of A~^T):  g = c~ - A~^T y, x^ = max(x - tau g, 0),
//                           x_bar = 2 x^ - x, x <- Halpern/reflection update
//   dual   (rows of A~):    y^ = y + sigma (b~ - A~ x_bar), y <- same update
// and at the end of a block of iterations: two float64 evaluation kernels, a
// single-workgroup decide kernel (tests, restart, primal weight) that writes a
// device-resident control block, and a conditional restart copy.  Blocks are
// captured once into a hipGraph and replayed; the host reads one status word
// per block.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.h"
#include "panel.h"
#include "plain.h"

namespace mip {

enum : int32_t { ST_RUNNING = -1 };
enum : int32_t { F_FIRST = 1, F_EVAL = 2, F_HAT = 4 };

// ---------------------------------------------------------------------------
// small vector kernels
// ---------------------------------------------------------------------------

__global__ void k_fill(double* p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
__global__ void k_fill_t(T* p, int64_t n, T v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// partial sums of squares of a float64 vector, one slot per workgroup
__global__ __launch_bounds__(kBlock) void k_sumsq(const double* v, int64_t n, double* partials) {
    double s[1] = {0.0};
    double mx[1] = {0.0};
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        s[0] += v[i] * v[i];
    block_reduce_store<1, 0>(s, mx, partials + blockIdx.x);
}

// out[q] = fixed-order sum over G partial rows of width W (one workgroup)
__global__ __launch_bounds__(kBlock) void k_reduce_rows(const double* partials, int G, int W,
                                                        double* out) {
    __shared__ double sh[kBlock];
    for (int q = 0; q < W; ++q) {
        double s = 0.0;
        int g = threadIdx.x;
        for (; g + 7 * kBlock < G; g += 8 * kBlock) {  // 8 loads in flight, added in the same order
            double x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = partials[(int64_t)(g + u * kBlock) * W + q];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += x[u];
        }
        for (; g < G; g += kBlock) s += partials[(int64_t)g * W + q];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int st = kBlock / 2; st > 0; st >>= 1) {
            if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[q] = sh[0];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// scaling
// ---------------------------------------------------------------------------
// stat[r] = d_self[r] * (max or sum over the row of |a_rk| d_other[col_k]),
// i.e. the row's infinity norm (MAXMODE) or 1-norm of the currently scaled
// matrix D_r A D_c.
template <bool MAXMODE>
__global__ __launch_bounds__(kBlock) void k_scale_stat(TilePlan p, const int32_t* col, const double* val,
                                                       const double* d_self, const double* d_other,
                                                       double* stat) {
    extern __shared__ __align__(16) unsigned char smem_t[];
    const auto L = tile_lds<double>(smem_t, p);
    auto prod = [&](int b, int j) {
        const int64_t k = (int64_t)b + j;
        return fabs(val[k]) * d_other[col[k]];
    };
    auto epi = [&](int r, double a) { stat[r] = d_self[r] * a; };
    auto le = lepi(epi);
    tiled_rows<MAXMODE>(p, own_tile(), L, prod, le);
}

// d[i] *= 1/sqrt(stat[i]) (1 for an empty row or column)
__global__ void k_scale_update(double* d, const double* stat, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double s = stat[i];
        if (s > 0.0) d[i] = d[i] * (1.0 / sqrt(s));
    }
}

// part[b] = max of this block's grid-stride share of v (0 for none)
__global__ __launch_bounds__(kBlock) void k_max_part(const double* v, int64_t n, double* part) {
    __shared__ double sh[kBlock];
    double mx = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        mx = fmax(mx, v[i]);
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// out[k] = d_self[r] * val[k] * d_other[col[k]] rounded to V, for every row r
template <typename V>
__global__ __launch_bounds__(kBlock) void k_scale_values(const int32_t* rowptr, const int32_t* col,
                                                         const double* val, const double* d_self,
                                                         const double* d_other, int32_t nrows, V* out) {
    // one wave per row group of 64 lanes striding the row
    const int lane = threadIdx.x & (kWave - 1);
    for (int64_t r = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / kWave; r < nrows;
         r += (int64_t)gridDim.x * (kBlock / kWave)) {
        const int st = rowptr[r], e = rowptr[r + 1];
        const double ds = d_self[r];
        for (int k = st + lane; k < e; k += kWave) {
            double v = ds * val[k] * d_other[col[k]];
            if constexpr (sizeof(V) == 2) {
                out[k] = f32_to_bf16_rne((float)v);
            } else {
                out[k] = (V)v;
            }
        }
    }
}

template <typename V>
__device__ __forceinline__ void store_scaled(V* out, int64_t k, double v) {
    if constexpr (sizeof(V) == 2) {
        out[k] = f32_to_bf16_rne((float)v);
    } else {
        out[k] = (V)v;
    }
}

// Sorted tile layout of one scaled copy.  Inside every tile (one workgroup
// per tile) the nonzeros are ordered by column with an LDS bitonic sort of
// (column, position) keys, which are unique, so the order is deterministic.
// Written per sorted position k: the column, the 16-bit row-major position
// in the tile (slot), and the scaled value d_self[row] * val * d_other[col]
// in the iteration precision (the same expression as k_scale_values).  A
// tile holding one row longer than tile_nnz keeps the row-major order.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_sort_scale_tiles(TilePlan p, const int32_t* col, const double* val,
                                                             const double* d_self, const double* d_other,
                                                             int32_t* col_s, uint16_t* slot_s, V* out) {
    extern __shared__ __align__(16) unsigned char smem_t[];
    int pw = 1;
    while (pw < p.tile_nnz) pw <<= 1;
    unsigned long long* key = (unsigned long long*)smem_t;
    int32_t* rows = (int32_t*)(key + pw);
    const int tid = threadIdx.x;
    const int4 d = p.desc[blockIdx.x];
    const int r0 = d.x, nr = d.y - d.x, s = d.z, e = d.w, nz = e - s;
    if (nz > p.tile_nnz) {
        const double ds = d_self[r0];
        for (int k = s + tid; k < e; k += kBlock) {
            const int c = col[k];
            col_s[k] = c;
            slot_s[k] = 0;
            store_scaled(out, k, ds * val[k] * d_other[c]);
        }
        return;
    }
    int P = 1;
    while (P < nz) P <<= 1;
    for (int i = tid; i < P; i += kBlock)
        key[i] = i < nz ? ((unsigned long long)(uint32_t)col[s + i] << 16) | (unsigned)i : ~0ull;
    for (int i = tid; i <= nr; i += kBlock) rows[i] = p.rowptr[r0 + i] - s;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < P; i += kBlock) {
                const int l = i ^ j;
                if (l > i) {
                    const unsigned long long a = key[i], b = key[l];
                    if ((a > b) == ((i & k) == 0)) {
                        key[i] = b;
                        key[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    for (int i = tid; i < nz; i += kBlock) {
        const unsigned long long kv = key[i];
        const int c = (int)(kv >> 16), src = (int)(kv & 0xffffu);
        int lo = 0, hi = nr;  // rows[lo] <= src < rows[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (rows[mid] <= src) lo = mid;
            else hi = mid;
        }
        col_s[s + i] = c;
        slot_s[s + i] = (uint16_t)src;
        store_scaled(out, s + i, d_self[r0 + lo] * val[s + src] * d_other[c]);
    }
}

inline size_t sort_lds_bytes(const TilePlan& p) {
    size_t pw = 1;
    while (pw < (size_t)p.tile_nnz) pw <<= 1;
    return 8 * pw + 4 * (size_t)(p.tile_rows + 1);
}

// t[i] = d[i] * v[i] rounded to T (unless out is NULL); partial sums of
// squares in float64
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scale_vec(const double* v, const double* d, int64_t n,
                                                      T* out, double* partials) {
    double s[1] = {0.0};
    double mx[1] = {0.0};
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        double t = d[i] * v[i];
        if (out) out[i] = (T)t;
        s[0] += t * t;
    }
    block_reduce_store<1, 0>(s, mx, partials + blockIdx.x);
}

// ---------------------------------------------------------------------------
// power iteration on D_r A D_c, float64 vectors and sums
// ---------------------------------------------------------------------------
// y[r] = sum_k a~_k x[col[k]] over the iteration's scaled copy (values
// already D_r A D_c in the iteration precision, sorted or row-major tile
// layout), partial ||y||^2: the power iteration measures the matrix the
// iteration actually applies, with one gather per nonzero (scaling the
// float64 original on the fly would gather the column factor as well).
// Products and sums in float64.
// The power iteration's SpMV on the scaled copy: vectors of type X (the
// iterate type: float64, or float32 in the FP32 modes, whose scaled matrix is
// itself rounded to float32 or BF16), products and row sums in float64.
template <typename V, bool SORTED, typename X, int U>
__global__ __launch_bounds__(kBlock) void k_spmv_copy(TilePlan p, const int32_t* col, const V* vals,
                                                      const X* x, X* y, double* partials) {
    extern __shared__ __align__(16) unsigned char smem_t[];
    const auto L = tile_lds<double>(smem_t, p);
    double s[1] = {0.0};
    double mx[1] = {0.0};
    auto prod = [&](int b, int j) {
        return (double)ld_val_at(vals + b, j) * (double)x[ld_at_nt(col + b, j)];
    };
    auto epi = [&](int r, double a) {
        y[r] = (X)a;
        s[0] += a * a;
    };
    auto le = lepi(epi);
    tiled_rows<false, double, U, SORTED>(p, own_tile(), L, prod, le);
    block_reduce_store<1, 0>(s, mx, partials + blockIdx.x);
}

// v = u / sqrt(sum of G partials), identical sum order in every workgroup
template <typename X>
__global__ __launch_bounds__(kBlock) void k_normalize(const X* u, X* v, int64_t n,
                                                      const double* partials, int G) {
    __shared__ double sh[kBlock];
    double s = 0.0;
    for (int g = threadIdx.x; g < G; g += kBlock) s += partials[g];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    const double nrm = sqrt(sh[0]);
    if (nrm == 0.0) return;  // u = 0: keep v
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        v[i] = (X)((double)u[i] / nrm);
}

// ---------------------------------------------------------------------------
// iteration kernels
// ---------------------------------------------------------------------------
// Iterates are held relative to the epoch's anchor (x0, y0): the state is
// u = x - x0, v = y - y0, the extrapolation x_bar - x0, and the right-hand
// sides are the anchor's residuals r_c = c~ - A~^T y0, r_b = b~ - A~ x0,
// formed in float64 with the caller's matrix at every restart.  So
// g = c~ - A~^T y = r_c - A~^T v and b~ - A~ x_bar = r_b - A~ (x_bar - x0):
// the stored matrix and vectors only ever carry the epoch's movement, and
// in reduced precision their rounding errors are relative to it (not to the
// iterate).  The projected points x^, y^ are stored absolute.
template <typename T, typename V>
struct IterArgs {
    RowPlan p;
    const int32_t* col;
    const V* val;
    const T* gather;   // v (primal) or x_bar - x0 (dual)
    T* state;          // u or v
    T* bar;            // x_bar - x0 (primal only)
    T* hat;            // x^ or y^ (absolute)
    const T* anchor;   // Halpern anchor x0 or y0
    const T* rhs;      // r_c or r_b
    double* out64;     // x or y of the original model, written at evaluations
    const double* dscale;  // D_c or D_r
    double* partials;  // [G][3]: ||o - h||^2 at the first iteration, same at the evaluation, ||h - anchor||^2
    const Ctrl* ctrl;
    const T* lo;          // general form, primal: scaled bounds l / D_c, u / D_c
    const T* hi;
    const int8_t* sense;  // general form, dual: row senses
    T* avg;               // restart to average: the epoch's mean of x^ or y^
    T* state_out;         // where the new u or v goes (the state itself, or with the
                          // adaptive step the other buffer of the pair)
    const T* ax_in;       // adaptive step, dual: A~ (x - x0) of the current iterate
    T* ax_out;            // and of the attempt's x^ (A~ (x - x0) + A~ (x^ - x))
    double* apart;        // adaptive step: per-block sums of the attempt's move
    double rho;
    int32_t halpern;
    int32_t it;
    int32_t flags;
};

// Per-row epilogue of the primal (PRIMAL) or dual step, shared by both SpMV
// traversals.  q accumulates the three partial sums described in IterArgs.
// load() fetches the row's vector entries ahead of the SpMV; apply() finishes.
template <typename T>
struct IterPre {
    T o, an, rhs;
    T lo, hi;  // general form, primal
    int sense; // general form, dual
    T av;      // restart to average
    T ax;      // adaptive step, dual: A~ (x - x0)
};

// GEN: the general form (Section 2 mentions bounds and inequality rows):
// the primal step projects onto [l, u] instead of x >= 0, the dual step
// keeps y_i >= 0 on >= rows and y_i <= 0 on <= rows.
// AVG: restart to average: the epoch's running mean of the projected points
// is updated (avg = h after the epoch's first iteration, avg += (h - avg) / j
// after its j-th) and its distance to the anchor replaces that of h in the
// evaluation partials.
// ADAPT: the adaptive step (plain PDHG, no Halpern, no reflection): the
// primal hands the dual the move x^ - x instead of x_bar - x0, so that the
// dual's row sum is A~ (x^ - x) itself (no cancellation in the step rule's
// cross term); the dual forms A~ (x_bar - x0) = A~ (x - x0) + 2 A~ (x^ - x)
// from the kept product of the current iterate, keeps A~ (x^ - x0) for the
// next attempt, and both add the move's terms ||x^ - x||^2 (q[3]),
// ||y^ - y||^2 (q[3]) and (y^ - y)^T A~ (x^ - x) (q[4]).
template <typename T, typename V, bool PRIMAL, bool GEN, bool AVG = false, bool ADAPT = false>
struct IterEpi {
    const IterArgs<T, V>& a;
    double w, omw, rho, opr, st;
    int flags;
    double* q;
    bool run;
    double inv_j = 1.0;
    typedef IterPre<T> Pre;
    // The run flag, the Halpern weight and the step come from the device
    // control block; they are read here, once the tile's independent loads
    // are in flight.
    __device__ __forceinline__ bool running() const { return run; }
    __device__ __forceinline__ void ready() {
        const Ctrl* c = a.ctrl;
        run = c->status == ST_RUNNING;
        const int64_t k = c->k_base + a.it;
        w = a.halpern ? (double)(k + 1) / (double)(k + 2) : 1.0;
        omw = 1.0 - w;
        st = PRIMAL ? c->tau : c->sigma;
        if (AVG) inv_j = k == 0 ? 0.0 : 1.0 / (double)(k + 1);  // 0: the epoch's first point
    }
    // branch-free, so that the loads of all rows of a thread are in flight
    // together (the scaling factor is fetched by apply() on evaluations only)
    __device__ __forceinline__ Pre load(int r0, int i) const {
        Pre p;
        p.o = ld_at(a.state + r0, i);
        // the dual needs its anchor only to project (general form), to
        // average, or to form y^ at stored iterations
        p.an = (PRIMAL || GEN || AVG || (flags & F_HAT)) ? ld_at(a.anchor + r0, i) : (T)0;
        p.rhs = ld_at(a.rhs + r0, i);
        if (GEN && PRIMAL) {
            p.lo = ld_at(a.lo + r0, i);
            p.hi = ld_at(a.hi + r0, i);
        }
        if (GEN && !PRIMAL) p.sense = ld_at(a.sense + r0, i);
        if (AVG) p.av = ld_at(a.avg + r0, i);
        if (ADAPT && !PRIMAL) p.ax = ld_at(a.ax_in + r0, i);
        return p;
    }
    // The arithmetic is float64 whatever the storage type T: the stored
    // iterates are rounded once, at the store.  dh is the projected point
    // relative to the anchor (x^ - x0 or y^ - y0).
    template <typename Acc>
    __device__ __forceinline__ void apply(int r0, int i, const Pre& p, Acc s) const {
        const double o = (double)p.o;    // u or v
        const double an = (double)p.an;  // x0 or y0 (0 where the dual did not load it)
        double dh;
        if (PRIMAL) {
            const double g = (double)p.rhs - (double)s;  // c~ - A~^T y
            dh = o - st * g;
            if (GEN) {  // projection of x0 + dh onto [l, u] (NaN propagates)
                const double l = (double)p.lo - an, u = (double)p.hi - an;
                dh = dh < l ? l : (dh > u ? u : dh);
            } else {
                dh = dh < -an ? -an : dh;  // projection onto x >= 0 (NaN propagates)
            }
            st_at(a.bar + r0, i, (T)(ADAPT ? dh - o : 2.0 * dh - o));
            if (ADAPT) q[3] += (dh - o) * (dh - o);
        } else {
            double sb = (double)s;
            if (ADAPT) {  // s = A~ (x^ - x): extrapolate from the kept A~ (x - x0)
                const double ax = (double)p.ax;
                sb = ax + 2.0 * (double)s;
                st_at(a.ax_out + r0, i, (T)(ax + (double)s));
            }
            dh = o + st * ((double)p.rhs - sb);  // v + sigma (b~ - A~ x_bar)
            if (GEN) {  // the sign each row's sense allows y0 + dh
                if (p.sense == MIPDHG_SENSE_GE) dh = dh < -an ? -an : dh;
                else if (p.sense == MIPDHG_SENSE_LE) dh = dh > -an ? -an : dh;
            }
            if (ADAPT) {
                const double dy = dh - o;
                q[3] += dy * dy;
                q[4] += dy * (double)s;
            }
        }
        const double h = an + dh;  // x^ or y^
        if (flags & F_HAT) st_at(a.hat + r0, i, (T)h);
        // Halpern/reflection step; the anchor is 0 in these coordinates
        st_at(a.state_out + r0, i, (T)(w * (opr * dh - rho * o)));
        double rd = dh;  // the restart point's distance to the anchor
        if (AVG) {  // the epoch's mean; its first point is taken as it is (the buffer is not read)
            double rp = h;
            if (inv_j != 0.0) {
                const double av = (double)p.av;
                rp = av + (h - av) * inv_j;
            }
            st_at(a.avg + r0, i, (T)rp);
            rd = rp - an;
        }
        if (flags & (F_FIRST | F_EVAL)) {
            double d = o - dh;
            d *= d;
            if (flags & F_FIRST) q[0] += d;
            if (flags & F_EVAL) q[1] += d;
        }
        if (flags & F_EVAL) {
            q[2] += rd * rd;
            st_at(a.out64 + r0, i, ld_at(a.dscale + r0, i) * h);
        }
    }
    // lane-group traversal: load and apply at once
    template <typename Acc>
    __device__ __forceinline__ void operator()(int r, Acc s) const {
        apply(r, 0, load(r, 0), s);
    }
};

template <typename T, typename V, bool PRIMAL, bool GEN = false, bool AVG = false, bool ADAPT = false>
__device__ __forceinline__ IterEpi<T, V, PRIMAL, GEN, AVG, ADAPT> make_epi(const IterArgs<T, V>& a, double* q) {
    IterEpi<T, V, PRIMAL, GEN, AVG, ADAPT> e{a, 1.0, 0.0, a.rho, 1.0 + a.rho, 0.0, a.flags, q, false};
    return e;
}

__device__ __forceinline__ unsigned iter_store_mask(int flags) {
    // slot 0 belongs to the block's first iteration, slots 1-2 to its evaluation
    return ((flags & F_FIRST) ? 1u : 0u) | ((flags & F_EVAL) ? 6u : 0u);
}

// lane-group traversal (RowPlan); SpMV accumulated in Acc
template <typename T, typename V, typename Acc, int L, bool PRIMAL>
__global__ __launch_bounds__(kBlock) void k_iter(IterArgs<T, V> a) {
    if (a.ctrl->status != ST_RUNNING) return;
    double q[3] = {0.0, 0.0, 0.0};
    double mx[1] = {0.0};
    auto epi = make_epi<T, V, PRIMAL>(a, q);
    epi.ready();
    auto dot = [&](int s, int e, int lane, int LL) {
        Acc acc = 0;
#pragma unroll 4
        for (int kk = s + lane; kk < e; kk += LL) acc += ld_val(a.val, kk) * (Acc)a.gather[ld_idx(a.col, kk)];
        return acc;
    };
    for_rows<L, Acc>(a.p, dot, epi);
    if (a.flags & (F_FIRST | F_EVAL)) block_reduce_store<3, 0>(q, mx, a.partials + 3 * blockIdx.x, iter_store_mask(a.flags));
}

// LDS-tiled traversal (TilePlan).  The control word is loaded up front and
// only checked once the products are in LDS.
template <typename T, typename V, typename Acc, bool PRIMAL, int U, bool SORTED, bool GEN, bool AVG = false,
          bool ADAPT = false>
__global__ __launch_bounds__(kBlock) void k_iter_tiled(IterArgs<T, V> a, TilePlan tp) {
    // blocks queued behind the one that ended the solve stream nothing
    if (a.ctrl->status != ST_RUNNING) return;
    extern __shared__ __align__(16) unsigned char smem_t[];
    const auto L = tile_lds<Acc>(smem_t, tp);
    double q[ADAPT ? 5 : 3] = {};
    double mx[1] = {0.0};
    auto epi = make_epi<T, V, PRIMAL, GEN, AVG, ADAPT>(a, q);
    // streamed arrays: tile base + 32-bit offset; the gather: a plain 64-bit
    // address, measured 12-18 % faster than the base + offset form on
    // 4096- and 8192-nonzero tiles
    auto prod = [&](int b, int j) {
        return ld_val_at(a.val + b, j) * (Acc)a.gather[(int64_t)ld_at_nt(a.col + b, j)];
    };
    tiled_rows<false, Acc, U, SORTED>(tp, own_tile(), L, prod, epi);
    if (epi.running() && (a.flags & (F_FIRST | F_EVAL))) {
        if constexpr (ADAPT) {
            double q3[3] = {q[0], q[1], q[2]};
            block_reduce_store<3, 0>(q3, mx, a.partials + 3 * blockIdx.x, iter_store_mask(a.flags));
        } else {
            block_reduce_store<3, 0>(q, mx, a.partials + 3 * blockIdx.x, iter_store_mask(a.flags));
        }
    }
    if constexpr (ADAPT) {
        if (epi.running()) {
            constexpr int NA = PRIMAL ? 1 : 2;
            double qa[NA];
            qa[0] = q[3];
            if (!PRIMAL) qa[NA - 1] = q[4];
            block_reduce_store<NA, 0>(qa, mx, a.apart + NA * blockIdx.x);
        }
    }
}

// The same step as a persistent launch: about one workgroup per resident slot,
// each walking its XCD's run of tiles, so that no time goes to dispatching a
// workgroup per tile.  The norm partials cover all tiles of a workgroup.
template <typename T, typename V, typename Acc, bool PRIMAL, int U, bool SORTED, bool GEN>
__global__ __launch_bounds__(kBlock) void k_iter_persist(IterArgs<T, V> a, TilePlan tp) {
    if (a.ctrl->status != ST_RUNNING) return;
    extern __shared__ __align__(16) unsigned char smem_t[];
    const auto L = tile_lds<Acc>(smem_t, tp);
    double q[3] = {0.0, 0.0, 0.0};
    double mx[1] = {0.0};
    auto epi = make_epi<T, V, PRIMAL, GEN>(a, q);
    auto prod = [&](int b, int j) {
        return ld_val_at(a.val + b, j) * (Acc)a.gather[(int64_t)ld_at_nt(a.col + b, j)];
    };
    const TileRange tr = persistent_tiles(tp.ntiles);
    for (int t = tr.first; t < tr.end; t += tr.step) {
        tiled_rows<false, Acc, U, SORTED>(tp, t, L, prod, epi);
        if (!epi.running()) return;
        __syncthreads();  // the next tile reuses the LDS
    }
    if (a.flags & (F_FIRST | F_EVAL))
        block_reduce_store<3, 0>(q, mx, a.partials + 3 * blockIdx.x, iter_store_mask(a.flags));
}

// ---------------------------------------------------------------------------
// dual step on the panel layout (panel.h)
// ---------------------------------------------------------------------------
typedef float pf4 __attribute__((ext_vector_type(4)));
typedef double pd2 __attribute__((ext_vector_type(2)));
typedef unsigned pu4 __attribute__((ext_vector_type(4)));

template <typename T, typename V>
struct PanelArgs {
    int32_t width;     // panel width, a power of two <= panel_width<T>()
    const PanelGroup* groups;
    const PanelUnit* units;
    const PanelChunk* chunks;
    const V* val;
    const uint16_t* col;
    const uint16_t* rid;
    const T* gather;   // x_bar - x0
    T* partial;
    int64_t ncols;
    const Ctrl* ctrl;
};

// A chunk's raw loads for one lane: 8 values, 8 columns, 8 row indices.
template <typename V>
struct PanelRaw;
template <>
struct PanelRaw<float> {
    pf4 v0, v1;
    pu4 col, rid;
    __device__ __forceinline__ void load(const float* v, const uint16_t* c, const uint16_t* r) {
        v0 = __builtin_nontemporal_load((const pf4*)v);
        v1 = __builtin_nontemporal_load((const pf4*)(v + 4));
        col = __builtin_nontemporal_load((const pu4*)c);
        rid = __builtin_nontemporal_load((const pu4*)r);
    }
    __device__ __forceinline__ double val(int j) const { return j < 4 ? v0[j] : v1[j - 4]; }
};
template <>
struct PanelRaw<double> {
    pd2 v[4];
    pu4 col, rid;
    __device__ __forceinline__ void load(const double* p, const uint16_t* c, const uint16_t* r) {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = __builtin_nontemporal_load((const pd2*)(p + 2 * q));
        col = __builtin_nontemporal_load((const pu4*)c);
        rid = __builtin_nontemporal_load((const pu4*)r);
    }
    __device__ __forceinline__ double val(int j) const { return v[j >> 1][j & 1]; }
};
template <>
struct PanelRaw<uint16_t> {  // BF16 values, widened exactly
    pu4 v, col, rid;
    __device__ __forceinline__ void load(const uint16_t* p, const uint16_t* c, const uint16_t* r) {
        v = __builtin_nontemporal_load((const pu4*)p);
        col = __builtin_nontemporal_load((const pu4*)c);
        rid = __builtin_nontemporal_load((const pu4*)r);
    }
    __device__ __forceinline__ double val(int j) const {
        const unsigned w = v[j >> 1];
        return (double)__uint_as_float((j & 1) ? (w & 0xffff0000u) : (w << 16));
    }
};
__device__ __forceinline__ int u16_at(const pu4& w, int j) {
    return (int)((j & 1) ? (w[j >> 1] >> 16) : (w[j >> 1] & 0xffffu));
}

// Stages gather[c0 .. c0 + len) into xs[x0 ..) (zero past ncols): every
// 16-byte load of a thread issued before its LDS writes.  c0 and x0 are
// multiples of 8 elements.
template <typename T>
__device__ __forceinline__ void panel_stage(T* xs, int x0, const T* gather, int64_t c0, int len, int64_t ncols) {
    constexpr int kVec = 16 / (int)sizeof(T);
    typedef T VT __attribute__((ext_vector_type(kVec)));
    constexpr int kPer = panel_width<T>() / (kPanelBlock * kVec);
    VT buf[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int i = (k * kPanelBlock + (int)threadIdx.x) * kVec;
        if (i < len) {
            const int64_t c = c0 + i;
            if (c + kVec <= ncols) {
                buf[k] = *(const VT*)(gather + c);
            } else {
#pragma unroll
                for (int e = 0; e < kVec; ++e) buf[k][e] = c + e < ncols ? gather[c + e] : (T)0;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int i = (k * kPanelBlock + (int)threadIdx.x) * kVec;
        if (i < len) *(VT*)&xs[x0 + i] = buf[k];
    }
}

// The waves of the workgroup take chunks c0 + wave, c0 + wave + 16, ... of
// up to 512 nonzeros, 8 per lane (vector loads, the next chunk's issued
// before the current one is summed), and sum each row's products with the
// staged vector xs in float64 in the row order of the matrix: a lane adds its
// own run of elements, a segmented scan over the lanes adds the runs of rows
// that cross lanes, and the lane holding a row's last element calls
// emit(global row, sum).  W: the staged width (a power of two).
// body: fetch(chunk) as soon as the chunk's descriptor is known (a chunk
// ahead of its processing), begin(chunk) when its processing starts,
// emit(row, sum), end(chunk).
template <typename T, typename V, typename Body>
__device__ __forceinline__ void panel_chunks(const PanelChunk* chunks, int32_t c_begin, int32_t c_end, const V* valp,
                                             const uint16_t* colp, const uint16_t* ridp, const T* xs, int W,
                                             Body& body) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    constexpr int kStride = kPanelBlock / kWave;
    int c = c_begin + wave;
    PanelChunk ch{0, 0, 0, 0};
    PanelRaw<V> raw;
    if (c < c_end) {
        ch = chunks[c];
        if (ch.count > lane * 8) {
            const int64_t e0 = (int64_t)ch.start + lane * 8;
            raw.load(valp + e0, colp + e0, ridp + e0);
        }
        body.fetch(ch);
    }
    for (; c < c_end; c += kStride) {
        const PanelChunk cur = ch;
        const PanelRaw<V> rc = raw;
        body.begin(cur);
        if (c + kStride < c_end) {  // the next chunk's loads go out first
            ch = chunks[c + kStride];
            if (ch.count > lane * 8) {
                const int64_t e0 = (int64_t)ch.start + lane * 8;
                raw.load(valp + e0, colp + e0, ridp + e0);
            }
            body.fetch(ch);
        }
        const int n = cur.count - lane * 8;  // this lane's elements (may be <= 0 or > 8)
        int rr[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) rr[j] = n > 0 ? u16_at(rc.rid, j) : -1;
        double s[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const double pr = j < n ? rc.val(j) * (double)xs[u16_at(rc.col, j) & (W - 1)] : 0.0;
            s[j] = (j > 0 && rr[j] == rr[j - 1]) ? s[j - 1] + pr : pr;
        }
        // the run ending at element 7 starts in this lane unless element 0
        // continues the previous lane's last row and no row starts after it
        const int prev_r7 = __shfl_up(rr[7], 1, kWave);
        const bool cont0 = lane > 0 && rr[0] == prev_r7;
        bool starts = !cont0;
#pragma unroll
        for (int j = 1; j < 8; ++j) starts = starts || rr[j] != rr[j - 1];
        // inclusive segmented scan of the runs over the lanes (earlier on the left)
        double inc = s[7];
        int f = starts ? 1 : 0;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const double t2 = __shfl_up(inc, d, kWave);
            const int f2 = __shfl_up(f, d, kWave);
            if (lane >= d) {
                if (!f) inc = t2 + inc;
                f |= f2;
            }
        }
        double carry = __shfl_up(inc, 1, kWave);
        if (!cont0) carry = 0.0;
        const int next_r0 = __shfl_down(rr[0], 1, kWave);
        const int next_n = __shfl_down(n, 1, kWave);
        bool head = true;  // element j still in the row of element 0
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (j >= n) break;
            head = head && rr[j] == rr[0];
            const bool last = (j == 7) ? (lane == kWave - 1 || next_n <= 0 || next_r0 != rr[7])
                                       : (j + 1 >= n || rr[j + 1] != rr[j]);
            if (last) body.emit(cur.row0 + rr[j], s[j] + (head ? carry : 0.0));
        }
        body.end(cur);
    }
}

// One workgroup per unit: the panel's slice of the gathered vector is staged
// in LDS, then the unit's chunks are summed (panel_chunks) and each row's sum
// over the panel goes to its partial.
template <typename T, typename V>
__global__ __launch_bounds__(kPanelBlock) void k_panel_spmv(PanelArgs<T, V> a) {
    if (a.ctrl->status != ST_RUNNING) return;
    __shared__ __align__(16) T xs[panel_width<T>()];
    const int W = a.width;
    const PanelUnit un = a.units[blockIdx.x];
    const PanelGroup g = a.groups[un.group];
    const int64_t c0 = (int64_t)g.lo + (int64_t)un.panel * W;  // a multiple of 8
    panel_stage<T>(xs, 0, a.gather, c0, W, a.ncols);
    __syncthreads();
    struct Body {
        T* partial;
        __device__ __forceinline__ void fetch(const PanelChunk&) {}
        __device__ __forceinline__ void begin(const PanelChunk&) {}
        __device__ __forceinline__ void emit(int32_t r, double sum) { partial[r] = (T)sum; }
        __device__ __forceinline__ void end(const PanelChunk&) {}
    } body{a.partial + g.seg_base + (int64_t)un.panel * (g.r1 - g.r0) - g.r0};
    panel_chunks<T, V>(a.chunks, un.c0, un.c1, a.val, a.col, a.rid, xs, W, body);
}

template <typename V>
struct RowPanelArgs {
    int32_t width;
    const RowPanelGroup* groups;
    const RowPanelUnit* units;
    const PanelChunk* chunks;
    const V* val;
    const uint16_t* col;
    const uint16_t* rid;
    int32_t t0, tail;
    int64_t ncols;
};

// The primal step on A^T's row-panel layout: a workgroup per unit stages its
// group's window of v and the common tail in LDS and sums every row of the
// unit whole (panel_chunks).  A row-panel chunk holds at most
// kRowPanelChunkRows rows, its row count in the descriptor's last field: a
// chunk ahead of its processing, lane l issues the epilogue loads of the
// chunk's rows l and l + 64 (consecutive rows on consecutive lanes); the row
// sums go to the wave's slice of LDS; then each lane finishes its rows.
template <typename T, typename V, bool GEN>
__global__ __launch_bounds__(kPanelBlock) void k_rowpanel_primal(IterArgs<T, V> a, RowPanelArgs<V> pa) {
    if (a.ctrl->status != ST_RUNNING) return;
    __shared__ __align__(16) T xs[panel_width<T>()];
    __shared__ double rsum[kPanelBlock / kWave][kRowPanelChunkRows];
    double q[3] = {0.0, 0.0, 0.0};
    double mx[1] = {0.0};
    auto epi = make_epi<T, V, true, GEN>(a, q);
    epi.ready();
    const RowPanelUnit un = pa.units[blockIdx.x];
    const RowPanelGroup g = pa.groups[un.group];
    panel_stage<T>(xs, 0, a.gather, g.lo, g.ml, pa.t0);
    panel_stage<T>(xs, g.ml, a.gather, pa.t0, pa.tail, pa.ncols);
    __syncthreads();
    typedef typename decltype(epi)::Pre Pre;
    constexpr int kPer = kRowPanelChunkRows / kWave;
    struct Body {
        decltype(epi)& epi;
        double* rs;  // the wave's row sums, by row inside the chunk
        int lane;
        int32_t row0 = 0;
        Pre pre[kPer], nxt[kPer];
        __device__ __forceinline__ void fetch(const PanelChunk& ch) {
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int j = lane + k * kWave;
                if (j < ch.unit) nxt[k] = epi.load(ch.row0 + j, 0);
            }
        }
        __device__ __forceinline__ void begin(const PanelChunk& ch) {
            row0 = ch.row0;
#pragma unroll
            for (int k = 0; k < kPer; ++k) pre[k] = nxt[k];
        }
        __device__ __forceinline__ void emit(int32_t r, double sum) { rs[r - row0] = sum; }
        __device__ __forceinline__ void end(const PanelChunk& ch) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int j = lane + k * kWave;
                if (j < ch.unit) epi.apply(ch.row0 + j, 0, pre[k], rs[j]);
            }
            __builtin_amdgcn_wave_barrier();  // the next chunk's sums overwrite rs
        }
    };
    const int wave = threadIdx.x / kWave;
    Body body{epi, &rsum[wave][0], (int)(threadIdx.x & (kWave - 1))};
    panel_chunks<T, V>(pa.chunks, un.c0, un.c1, pa.val, pa.col, pa.rid, xs, pa.width, body);
    if (a.flags & (F_FIRST | F_EVAL))
        block_reduce_store<3, 0, kPanelBlock>(q, mx, a.partials + 3 * blockIdx.x, iter_store_mask(a.flags));
}

struct PanelRows {
    const PanelGroup* groups;
    const int32_t* row_group;
    const int32_t* wide_rows;  // rows of groups with more than kPanelRowsSerial panels
    int32_t nrows, nwide;
};

// Each row's partial sums added in a fixed order, then the dual epilogue.
// The first workgroups take one row per thread, adding a row's panels in
// panel order; rows of groups with more than kPanelRowsSerial panels
// (linking rows) are left to the last workgroups, where a wave takes one such
// row: lane l adds panels l, l + 64, ..., then a fixed butterfly tree adds
// the lanes and lane 0 finishes the row.
constexpr int kPanelRowsSerial = kPanelWideRow;

template <typename T, typename V, bool GEN>
__global__ __launch_bounds__(kBlock) void k_panel_rows(IterArgs<T, V> a, PanelRows pr, const T* partial) {
    if (a.ctrl->status != ST_RUNNING) return;
    double q[3] = {0.0, 0.0, 0.0};
    double mx[1] = {0.0};
    auto epi = make_epi<T, V, false, GEN>(a, q);
    epi.ready();
    const int nb = (pr.nrows + kBlock - 1) / kBlock;
    if ((int)blockIdx.x < nb) {
        const int r = blockIdx.x * kBlock + threadIdx.x;
        if (r < pr.nrows) {
            const PanelGroup g = pr.groups[pr.row_group[r]];
            if (g.np <= kPanelRowsSerial) {
                const int64_t R = g.r1 - g.r0;
                double sum = 0.0;
                for (int p = 0; p < g.np; ++p) sum += (double)partial[g.seg_base + p * R + (r - g.r0)];
                epi.apply(r, 0, epi.load(r, 0), sum);
            }
        }
    } else {
        const int lane = threadIdx.x & (kWave - 1);
        const int w = ((int)blockIdx.x - nb) * (kBlock / kWave) + (int)(threadIdx.x / kWave);
        if (w < pr.nwide) {
            const int r = pr.wide_rows[w];
            const PanelGroup g = pr.groups[pr.row_group[r]];
            const int64_t R = g.r1 - g.r0, off = g.seg_base + (r - g.r0);
            double v = 0.0;
            for (int p = lane; p < g.np; p += kWave) v += (double)partial[off + p * R];
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
            if (lane == 0) epi.apply(r, 0, epi.load(r, 0), v);
        }
    }
    if (a.flags & (F_FIRST | F_EVAL))
        block_reduce_store<3, 0>(q, mx, a.partials + 3 * blockIdx.x, iter_store_mask(a.flags));
}

// ---------------------------------------------------------------------------
// evaluation on the original model (float64), Section 2 and Section 4.3
// ---------------------------------------------------------------------------
// ROWS:  over A's rows, r_p = b - A x; partials: sum r_p^2, sum b.y, then
//        the certificate sums below, max |r_p|
// !ROWS: over A^T's rows, z = max(c - A^T y, 0), r_d = c - A^T y - z;
//        partials: sum r_d^2, sum c.x, sum x.z, sum of bound terms, the
//        certificate sums, max |r_d|
// Infeasibility certificates (rays): (d, e) = the change of (x, y) since the
// previous evaluation, whose A x, A^T y, x and y each kernel keeps per row
// (read, then overwritten by this evaluation's): A d = A x - (A x)_prev,
// A^T e = A^T y - (A^T y)_prev.  ROWS sums: (part of A d outside the row's
// recession cone)^2, b.e, (part of e outside the row's sign cone)^2.
// !ROWS sums, with g = -A^T e and mu = g projected onto the bound cones:
// (g - mu)^2, bound terms of mu, c.d, (part of d outside the bounds'
// recession cone)^2.
// GEN (general form): a row's r_p is the violating part of b - A x for its
// sense; z is c - A^T y projected onto the cone the bounds allow, the
// complementarity term is z^+ (x - l) + z^- (u - x) and the dual objective
// gains l z^+ - u z^- (finite bounds only; NULL lo means 0, NULL hi +inf).
struct EvalArgs {
    RowPlan p;
    const int32_t* col;
    const double* val;
    const double* gather;  // x (ROWS) or y
    const double* vec;     // b (ROWS) or c
    const double* own;     // y (ROWS) or x
    double* out1;          // r_p (ROWS) or z
    double* out2;          // r_d (!ROWS)
    double* partials;      // [G][kEvalRowsW] (ROWS) or [G][kEvalColsW]
    const Ctrl* ctrl;
    const int8_t* sense;   // GEN, ROWS
    const double* lo;      // GEN, !ROWS (nullable)
    const double* hi;      // GEN, !ROWS (nullable)
    double* prod_prev;     // rays: (A x)_prev (ROWS) or (A^T y)_prev, updated in place
    double* own_prev;      // rays: y_prev (ROWS) or x_prev, updated in place
    int32_t rays;          // 1: certificate sums
};
constexpr int kEvalRowsW = 6;  // 5 sums + max
constexpr int kEvalColsW = 9;  // 8 sums + max

template <bool ROWS, bool GEN>
__global__ __launch_bounds__(kBlock) void k_eval(EvalArgs a, TilePlan tp) {
    const bool active = a.ctrl->status == ST_RUNNING;
    if (!active) return;
    extern __shared__ __align__(16) unsigned char smem_t[];
    const auto L = tile_lds<double>(smem_t, tp);
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double mx[1] = {0.0};
    auto prod = [&](int b, int j) {
        const int64_t k = (int64_t)b + j;
        return ld_val(a.val, k) * a.gather[ld_idx(a.col, k)];
    };
    auto epi = [&](int r, double t) {
        const double v = a.vec[r];
        if (ROWS) {
            double rp = v - t;
            const int sn = GEN ? a.sense[r] : MIPDHG_SENSE_EQ;
            if (GEN) {
                if (sn == MIPDHG_SENSE_GE) rp = rp > 0.0 ? rp : 0.0;
                else if (sn == MIPDHG_SENSE_LE) rp = rp < 0.0 ? rp : 0.0;
            }
            if (a.rays) {
                const double own = a.own[r];
                const double td = t - a.prod_prev[r], e = own - a.own_prev[r];
                double vt = td, ve = 0.0;  // = rows: A d = 0, e free
                if (sn == MIPDHG_SENSE_GE) {
                    vt = td < 0.0 ? td : 0.0;
                    ve = e < 0.0 ? e : 0.0;
                } else if (sn == MIPDHG_SENSE_LE) {
                    vt = td > 0.0 ? td : 0.0;
                    ve = e > 0.0 ? e : 0.0;
                }
                s[2] += vt * vt;
                s[3] += v * e;
                s[4] += ve * ve;
                a.prod_prev[r] = t;
                a.own_prev[r] = own;
            }
            a.out1[r] = rp;
            s[0] += rp * rp;
            s[1] += v * a.own[r];
            mx[0] = fmax(mx[0], fabs(rp));
        } else {
            const double g = v - t;
            const double x = a.own[r];
            const double l = GEN && a.lo ? a.lo[r] : 0.0, u = GEN && a.hi ? a.hi[r] : INFINITY;
            const bool lf = isfinite(l), uf = isfinite(u);
            double z;
            if (GEN) {
                z = (lf && uf) ? g : lf ? (g > 0.0 ? g : 0.0) : uf ? (g < 0.0 ? g : 0.0) : 0.0;
                const double zp = z > 0.0 ? z : 0.0, zm = z < 0.0 ? -z : 0.0;
                s[2] += (lf ? zp * (x - l) : 0.0) + (uf ? zm * (u - x) : 0.0);
                s[3] += (lf ? l * zp : 0.0) - (uf ? u * zm : 0.0);
            } else {
                z = g > 0.0 ? g : 0.0;
                s[2] += x * z;
            }
            if (a.rays) {
                const double gr = -(t - a.prod_prev[r]), d = x - a.own_prev[r];
                double mu, vd;
                if (GEN) {
                    mu = (lf && uf) ? gr : lf ? (gr > 0.0 ? gr : 0.0) : uf ? (gr < 0.0 ? gr : 0.0) : 0.0;
                    vd = (lf && uf) ? d : lf ? (d < 0.0 ? d : 0.0) : uf ? (d > 0.0 ? d : 0.0) : 0.0;
                    const double mp = mu > 0.0 ? mu : 0.0, mm = mu < 0.0 ? -mu : 0.0;
                    s[5] += (lf ? l * mp : 0.0) - (uf ? u * mm : 0.0);
                } else {
                    mu = gr > 0.0 ? gr : 0.0;
                    vd = d < 0.0 ? d : 0.0;
                }
                s[4] += (gr - mu) * (gr - mu);
                s[6] += v * d;
                s[7] += vd * vd;
                a.prod_prev[r] = t;
                a.own_prev[r] = x;
            }
            const double rd = g - z;
            a.out1[r] = z;
            a.out2[r] = rd;
            s[0] += rd * rd;
            s[1] += v * x;
            mx[0] = fmax(mx[0], fabs(rd));
        }
    };
    auto le = lepi(epi);
    tiled_rows<false>(tp, own_tile(), L, prod, le, active);
    if (!active) return;
    if (ROWS) {
        double s5[5] = {s[0], s[1], s[2], s[3], s[4]};
        block_reduce_store<5, 1>(s5, mx, a.partials + kEvalRowsW * blockIdx.x);
    } else {
        block_reduce_store<8, 1>(s, mx, a.partials + kEvalColsW * blockIdx.x);
    }
}

// ---------------------------------------------------------------------------
// decide: tests, restart, primal weight (one workgroup)
// ---------------------------------------------------------------------------
struct DecideArgs {
    Ctrl* ctrl;
    const double* pp;  // primal partials [gp][3]
    const double* pd;  // dual partials [gd][3]
    const double* per; // eval rows [ger][kEvalRowsW]
    const double* pec; // eval cols [gec][kEvalColsW]
    int32_t gp, gd, ger, gec;
    int32_t nit;
};

// Every column of a [G][W] array of partials reduced in one pass: column q
// is summed (or, for q >= NS, maximised) over g = tid, tid + kBlock, ... by
// each thread, then by the same pairwise tree for every column, so the
// result does not depend on the launch and is the same for each column as a
// reduction of that column alone.
template <int W, int NS>
__device__ void fixed_cols(const double* p, int G, double (&out)[W], double (*sh)[kBlock]) {
    double v[W];
#pragma unroll
    for (int q = 0; q < W; ++q) v[q] = 0.0;
    // a thread's entries g, g + kBlock, ... in that order; U of them loaded at once
    constexpr int U = W > 4 ? 4 : 8;
    int g = threadIdx.x;
    for (; g + (U - 1) * kBlock < G; g += U * kBlock) {
        double x[U][W];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < W; ++q) x[u][q] = p[(int64_t)(g + u * kBlock) * W + q];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < W; ++q) v[q] = q < NS ? v[q] + x[u][q] : fmax(v[q], x[u][q]);
    }
    for (; g < G; g += kBlock) {
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const double x = p[(int64_t)g * W + q];
            v[q] = q < NS ? v[q] + x : fmax(v[q], x);
        }
    }
#pragma unroll
    for (int q = 0; q < W; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
#pragma unroll
            for (int q = 0; q < W; ++q)
                sh[q][threadIdx.x] = q < NS ? sh[q][threadIdx.x] + sh[q][threadIdx.x + st]
                                            : fmax(sh[q][threadIdx.x], sh[q][threadIdx.x + st]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < W; ++q) out[q] = sh[q][0];
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_decide(DecideArgs a) {
    Ctrl& c = *a.ctrl;
    if (c.status != ST_RUNNING) return;
    __shared__ double sh[kEvalColsW][kBlock];
    double vp[3], vd[3], vr[kEvalRowsW], vc[kEvalColsW];
    fixed_cols<3, 3>(a.pp, a.gp, vp, sh);
    fixed_cols<3, 3>(a.pd, a.gd, vd, sh);
    fixed_cols<kEvalRowsW, kEvalRowsW - 1>(a.per, a.ger, vr, sh);
    fixed_cols<kEvalColsW, kEvalColsW - 1>(a.pec, a.gec, vc, sh);
    const double px_first = vp[0], px_eval = vp[1], px_anchor = vp[2];
    const double py_first = vd[0], py_eval = vd[1], py_anchor = vd[2];
    const double rp2 = vr[0], dobj = vr[1], rp_inf = vr[kEvalRowsW - 1];
    const double rd2 = vc[0], pobj = vc[1], xz = vc[2], bterm = vc[3];  // bterm: 0 in the standard form
    const double rd_inf = vc[kEvalColsW - 1];
    // certificate quantities (see k_eval)
    const bool rays = c.infeas_tol > 0.0 && c.have_prev;
    const double q_e = vr[3] + vc[5], r_e2 = vc[4] + vr[4];
    const double q_d = vc[6], r_d2 = vr[2] + vc[7];
    if (threadIdx.x != 0) return;

    const double om = c.omega;
    const int64_t t_end = c.t_base + a.nit;
    const int64_t k_end = c.k_base + a.nit;
    if (c.k_base == 0) c.R0 = sqrt(om * px_first + py_first / om);
    const double R = sqrt(om * px_eval + py_eval / om);
    c.rp2 = rp2;
    c.rd2 = rd2;
    c.pobj = pobj;
    c.dobj = dobj + bterm;
    c.xz = xz;
    c.rp_inf = rp_inf;
    c.rd_inf = rd_inf;
    c.eval_t = t_end;
    c.last_R = R;
    c.last_nit = a.nit;
    const double rp = sqrt(rp2), rd = sqrt(rd2), gap = fabs(pobj - c.dobj);
    int32_t status = ST_RUNNING;
    if (!(isfinite(rp2) && isfinite(rd2) && isfinite(pobj) && isfinite(c.dobj))) {
        status = MIPDHG_NUMERICAL;
    } else if (rp <= c.eps * (1.0 + c.b_norm) && rd <= c.eps * (1.0 + c.c_norm) &&
               gap <= c.eps * (1.0 + fabs(pobj) + fabs(c.dobj))) {
        status = MIPDHG_OPTIMAL;
    } else if (rays && q_e > 0.0 && sqrt(r_e2) <= c.infeas_tol * q_e) {
        status = MIPDHG_PRIMAL_INFEASIBLE;
    } else if (rays && q_d < 0.0 && sqrt(r_d2) <= c.infeas_tol * -q_d) {
        status = MIPDHG_DUAL_INFEASIBLE;
    } else if (t_end >= c.max_iter) {
        status = MIPDHG_ITER_LIMIT;
    }
    c.t_base = t_end;
    if (status != ST_RUNNING) {
        c.status = status;
        c.restart_now = 0;
        return;
    }
    c.have_prev = 1;  // the evaluation kernels have kept this evaluation's point
    bool restart = false;
    if (c.do_restarts) {
        restart = (R <= c.beta_suff * c.R0) || (R <= c.beta_nec * c.R0 && R > c.R_prev) ||
                  ((double)k_end >= c.beta_art * (double)t_end);
    }
    if (restart) {
        const double dx = sqrt(px_anchor), dy = sqrt(py_anchor);
        if (dx > 1e-10 && dy > 1e-10) {
            const double th = c.pw_theta;
            if (c.pw_ki == 0.0 && c.pw_kd == 0.0) {
                c.omega = exp(th * log(dy / dx) + (1.0 - th) * log(c.omega));
            } else {
                const double e = log(c.omega) - log(dy / dx);
                c.pw_int += e;
                const double de = c.pw_count > 0 ? e - c.pw_err : 0.0;
                c.pw_err = e;
                c.pw_count += 1;
                c.omega = exp(log(c.omega) - (th * e + c.pw_ki * c.pw_int + c.pw_kd * de));
            }
            c.tau = c.eta / c.omega;
            c.sigma = c.eta * c.omega;
        }
        c.k_base = 0;
        c.R_prev = INFINITY;
        c.restarts += 1;
        c.restart_now = 1;
    } else {
        c.R_prev = R;
        c.k_base = k_end;
        c.restart_now = 0;
    }
}

// on a restart: anchor <- restart point, state (relative to it) <- 0, and
// with the adaptive step the kept A~ (x - x0) <- 0 (ax, else NULL)
template <typename T>
__global__ void k_apply_restart(const Ctrl* c, T* x, T* x0, const T* xh, int64_t n, T* y, T* y0,
                                const T* yh, int64_t m, T* ax) {
    if (!c->restart_now) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        x0[i] = xh[i];
        x[i] = (T)0;
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        y0[i] = yh[i];
        y[i] = (T)0;
        if (ax) ax[i] = (T)0;
    }
}

// ---------------------------------------------------------------------------
// adaptive step with rejection (the step rule of PDLP)
// ---------------------------------------------------------------------------
struct StepArgs {
    Ctrl* ctrl;
    const double* ap;  // [gp]: ||x^ - x||^2 per primal block
    const double* ad;  // [gd][2]: ||y^ - y||^2, (y^ - y)^T A~ (x^ - x) per dual block
    int gp, gd;
    int32_t it;        // the attempt's index in its block
};

// One workgroup: the move's sums in fixed order, then the rule: eta_bar =
// (omega ||dx||^2 + ||dy||^2 / omega) / (2 |dy^T A~ dx|) (infinite for a zero
// product); the attempt is accepted when eta <= eta_bar; the next step is
// min((1 - (t + 1)^-0.3) eta_bar, (1 + (t + 1)^-0.6) eta), t the attempt's
// 1-based number.
__global__ __launch_bounds__(kBlock) void k_step(StepArgs a) {
    Ctrl& c = *a.ctrl;
    if (c.status != ST_RUNNING) return;
    __shared__ double sh[2][kBlock];
    double vp[1], vd[2];
    fixed_cols<1, 1>(a.ap, a.gp, vp, sh);
    fixed_cols<2, 2>(a.ad, a.gd, vd, sh);
    if (threadIdx.x != 0) return;
    const double om = c.omega, eta = c.eta;
    const double mag = fabs(vd[1]);
    const double bar = mag > 0.0 ? (om * vp[0] + vd[0] / om) / (2.0 * mag) : INFINITY;
    const double t = (double)(c.t_base + a.it + 1);
    const double nxt = fmin((1.0 - pow(t + 1.0, -0.3)) * bar, (1.0 + pow(t + 1.0, -0.6)) * eta);
    const bool ok = eta <= bar;
    c.accepted = ok ? 1 : 0;
    if (!ok) c.rejected += 1;
    c.eta = nxt;
    c.tau = nxt / om;
    c.sigma = nxt * om;
}

template <typename T>
struct RestoreArgs {
    const Ctrl* ctrl;
    const T *u_in, *v_in, *ax_in;  // the attempt's inputs
    T *u_out, *v_out, *ax_out;     // and outputs
    const T *x0, *y0;
    T *xhat, *yhat;                // F_HAT: the projected points the solve reports
    double *xo, *yo;               // F_EVAL: the evaluated point, original space
    const double *d_col, *d_row;
    double *pp, *pd;               // F_EVAL: slot 2 of the evaluation partials
    int64_t n, m;
    int gp, gd;
    int flags;
};

// After a rejected attempt: the outputs take the inputs back (the iterate
// stays), and where the attempt stored its projected point for the solve
// (F_HAT) or for the evaluation (F_EVAL) the current iterate replaces it,
// with its distance to the anchor in the evaluation partials.  Block b
// handles the b-th of gp chunks of the columns and of gd chunks of the rows,
// one partial slot each.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adapt_restore(RestoreArgs<T> a) {
    if (a.ctrl->status != ST_RUNNING || a.ctrl->accepted) return;
    const int b = blockIdx.x;
    double q[1] = {0.0};
    double mx[1] = {0.0};
    if (b < a.gp) {
        const int64_t ch = (a.n + a.gp - 1) / a.gp, i0 = (int64_t)b * ch, i1 = min(a.n, i0 + ch);
        for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
            const T u = a.u_in[i];
            a.u_out[i] = u;
            const double h = (double)a.x0[i] + (double)u;
            if (a.flags & F_HAT) a.xhat[i] = (T)h;
            if (a.flags & F_EVAL) {
                a.xo[i] = a.d_col[i] * h;
                q[0] += (double)u * (double)u;
            }
        }
    }
    if (a.flags & F_EVAL) {
        if (b < a.gp) block_reduce_store<1, 0>(q, mx, a.pp + 3 * b + 2);
        __syncthreads();
        q[0] = 0.0;
    }
    if (b < a.gd) {
        const int64_t ch = (a.m + a.gd - 1) / a.gd, i0 = (int64_t)b * ch, i1 = min(a.m, i0 + ch);
        for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
            const T v = a.v_in[i];
            a.v_out[i] = v;
            a.ax_out[i] = a.ax_in[i];
            const double h = (double)a.y0[i] + (double)v;
            if (a.flags & F_HAT) a.yhat[i] = (T)h;
            if (a.flags & F_EVAL) {
                a.yo[i] = a.d_row[i] * h;
                q[0] += (double)v * (double)v;
            }
        }
    }
    if ((a.flags & F_EVAL) && b < a.gd) block_reduce_store<1, 0>(q, mx, a.pd + 3 * b + 2);
}

// dst <- src for the three arrays of an iterate (u, v, A~ (x - x0))
template <typename T>
__global__ void k_copy_iterate(const T* u, T* u2, int64_t n, const T* v, T* v2, const T* ax, T* ax2, int64_t m) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        u2[i] = u[i];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        v2[i] = v[i];
        ax2[i] = ax[i];
    }
}

// The anchor's residuals in float64 on the caller's matrix, rounded once to
// T: over A's rows r_b = D_r (b - A D_c x0), over A^T's rows
// r_c = D_c (c - A^T D_r y0) (d_self, d_other: the row and column factors of
// the matrix walked; anchor: the anchor of the other side).  Runs at setup
// (force) and after a restart.
// d_other * anchor in float64 (the factor k_anchor_resid gathers per
// nonzero), under the same gate
template <typename T>
__global__ void k_anchor_scale(const double* d, const T* anchor, int64_t n, double* out, const Ctrl* ctrl, int force) {
    if (!force && !ctrl->restart_now) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = d[i] * (double)anchor[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_anchor_resid(TilePlan tp, const int32_t* col, const double* val,
                                                         const double* d_self, const double* scaled_anchor,
                                                         const double* vec, T* out, const Ctrl* ctrl, int force) {
    if (!force && !ctrl->restart_now) return;
    extern __shared__ __align__(16) unsigned char smem_t[];
    const auto L = tile_lds<double>(smem_t, tp);
    auto prod = [&](int b, int j) {
        const int64_t k = (int64_t)b + j;
        return ld_val(val, k) * scaled_anchor[ld_idx(col, k)];
    };
    auto epi = [&](int r, double t) { out[r] = (T)(d_self[r] * (vec[r] - t)); };
    auto le = lepi(epi);
    tiled_rows<false>(tp, own_tile(), L, prod, le);
}

// general form: scaled bounds l / D_c and u / D_c (NULL lo: 0, NULL hi: +inf)
template <typename T>
__global__ void k_scale_bounds(const double* lo, const double* hi, const double* d, int64_t n, T* lo_t, T* hi_t) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        lo_t[j] = (T)(lo ? lo[j] / d[j] : 0.0);
        hi_t[j] = (T)(hi ? hi[j] / d[j] : (double)INFINITY);
    }
}

// initial point: anchor = projected point = init / d (or 0), state 0
template <typename T>
__global__ void k_init_state(const double* init, const double* d, int64_t n, T* s, T* s0, T* hat) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T v = init ? (T)(init[i] / d[i]) : (T)0;
        s[i] = (T)0;
        s0[i] = v;
        hat[i] = v;
    }
}

// dst = src (+ base): the absolute iterate from the anchor and the state
template <typename T>
__global__ void k_export(const T* src, const T* base, double* dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = base ? (double)base[i] + (double)src[i] : (double)src[i];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int pow2_round(double v) {
    int L = 2;
    while (L < 64 && (double)L * 1.5 < v) L *= 2;
    return L;
}

HostPlan make_plan(const std::vector<int32_t>& rowptr, int32_t nrows, int32_t lanes_opt, int32_t long_opt) {
    HostPlan hp;
    const double mean = nrows > 0 ? (double)(rowptr[nrows] - rowptr[0]) / nrows : 0.0;
    hp.lanes = lanes_opt > 0 ? lanes_opt : std::min(32, pow2_round(mean));
    hp.long_thresh = long_opt > 0 ? long_opt : std::max(128, 4 * hp.lanes);
    for (int32_t r = 0; r < nrows; ++r)
        if (rowptr[r + 1] - rowptr[r] > hp.long_thresh) hp.long_rows.push_back(r);
    const int gpb = kBlock / hp.lanes;
    const int64_t need = (nrows + gpb - 1) / gpb;
    hp.g_short = (int32_t)std::max<int64_t>(1, std::min<int64_t>(need, kMaxShortBlocks));
    int64_t chunk = (nrows + hp.g_short - 1) / hp.g_short;
    chunk = (chunk + gpb - 1) / gpb * gpb;
    hp.chunk = (int32_t)std::max<int64_t>(chunk, gpb);
    hp.g_short = (int32_t)std::max<int64_t>(1, (nrows + hp.chunk - 1) / hp.chunk);
    const int64_t nl = (int64_t)hp.long_rows.size();
    hp.g_long = nl ? (int32_t)std::min<int64_t>((nl + 3) / 4, kMaxLongBlocks) : 0;
    return hp;
}

RowPlan device_plan(const HostPlan& hp, const int32_t* rowptr, const int32_t* long_rows_dev, int32_t nrows) {
    RowPlan p;
    p.rowptr = rowptr;
    p.long_rows = long_rows_dev;
    p.nrows = nrows;
    p.nlong = (int32_t)hp.long_rows.size();
    p.long_thresh = hp.long_thresh;
    p.lanes = hp.lanes;
    p.chunk = hp.chunk;
    p.g_short = hp.g_short;
    p.g_long = hp.g_long;
    p.pad = 0;
    return p;
}

// Greedy cut of the rows into tiles of at most tile_nnz nonzeros and tile_rows
// rows (a row longer than tile_nnz is a tile by itself), then ordered for the
// hardware: workgroups b and b + 8 run on the same XCD, and xcd_virtual_block() gives each
// XCD a contiguous range of descriptor slots.  "Heavy" tiles (holding a row
// of more than kHeavyRow nonzeros, whose gathers reach far across the vector)
// are dealt round-robin over the XCDs, first in each XCD's range; the light
// tiles fill the remaining slots in row order, so each XCD gathers from a
// contiguous stretch of rows.
constexpr int32_t kHeavyRow = 256;

std::vector<int32_t> make_tile_desc(const std::vector<int32_t>& rowptr, int32_t nrows, int32_t tile_nnz,
                                    int32_t tile_rows) {
    std::vector<int32_t> bounds;
    std::vector<char> heavy;
    bounds.reserve((size_t)max_tiles(nrows, rowptr[nrows], tile_nnz, tile_rows) + 1);
    bounds.push_back(0);
    int32_t r = 0;
    while (r < nrows) {
        const int32_t len = rowptr[r + 1] - rowptr[r];
        if (len > tile_nnz) {
            bounds.push_back(r + 1);
            heavy.push_back(1);
            ++r;
            continue;
        }
        const int32_t start = r;
        int64_t nz = 0;
        bool h = false;
        while (r < nrows && r - start < tile_rows) {
            const int32_t l = rowptr[r + 1] - rowptr[r];
            if (l > tile_nnz || nz + l > tile_nnz) break;
            nz += l;
            h |= l > kHeavyRow;
            ++r;
        }
        bounds.push_back(r);
        heavy.push_back(h ? 1 : 0);
    }
    const int64_t G = (int64_t)heavy.size();
    const int64_t q = G / 8, rem = G % 8;
    std::vector<int64_t> start(9, 0), fill(8, 0);
    for (int x = 0; x < 8; ++x) start[x + 1] = start[x] + q + (x < rem ? 1 : 0);
    std::vector<int64_t> slot_of(G, -1);
    int64_t nh = 0;
    for (int64_t i = 0; i < G; ++i)
        if (heavy[i]) {
            const int x = (int)(nh++ % 8);
            slot_of[i] = start[x] + fill[x]++;
        }
    int x = 0;
    for (int64_t i = 0; i < G; ++i) {
        if (heavy[i]) continue;
        while (start[x] + fill[x] >= start[x + 1]) ++x;
        slot_of[i] = start[x] + fill[x]++;
    }
    std::vector<int32_t> desc(4 * G);
    for (int64_t i = 0; i < G; ++i) {
        int32_t* d = &desc[4 * slot_of[i]];
        d[0] = bounds[i];
        d[1] = bounds[i + 1];
        d[2] = rowptr[bounds[i]];
        d[3] = rowptr[bounds[i + 1]];
    }
    return desc;
}

// Tiles of the greedy cut (for the autotuner's CU-balanced candidates).
int64_t tile_count(const std::vector<int32_t>& rowptr, int32_t nrows, int32_t tile_nnz, int32_t tile_rows) {
    return (int64_t)(make_tile_desc(rowptr, nrows, tile_nnz, tile_rows).size() / 4);
}

// The descriptors must cover every row exactly once with matching nonzero
// ranges and respect the tile limits; checked on the host before any launch.
bool tile_desc_ok(const std::vector<int32_t>& desc, const std::vector<int32_t>& rowptr, int32_t nrows,
                  int32_t tile_nnz, int32_t tile_rows) {
    const size_t G = desc.size() / 4;
    std::vector<std::pair<int32_t, int32_t>> ranges(G);
    for (size_t t = 0; t < G; ++t) {
        const int32_t r0 = desc[4 * t], r1 = desc[4 * t + 1], s = desc[4 * t + 2], e = desc[4 * t + 3];
        if (r0 < 0 || r1 <= r0 || r1 > nrows || s != rowptr[r0] || e != rowptr[r1]) return false;
        if (r1 - r0 > tile_rows || (e - s > tile_nnz && r1 - r0 != 1)) return false;
        ranges[t] = {r0, r1};
    }
    std::sort(ranges.begin(), ranges.end());
    int32_t next = 0;
    for (const auto& rg : ranges) {
        if (rg.first != next) return false;
        next = rg.second;
    }
    return next == nrows;
}

int32_t tile_nnz_of(const mipdhg_options& o) { return o.tile_nnz > 0 ? o.tile_nnz : kTileNnzDefault; }
int32_t tile_rows_of(const mipdhg_options& o) { return o.tile_rows > 0 ? o.tile_rows : kTileRowsDefault; }
int32_t short_row_of(const mipdhg_options& o) { return o.short_row != 0 ? o.short_row : kShortRowDefault; }
int32_t tile_nnz_at_of(const mipdhg_options& o) { return o.tile_nnz_at > 0 ? o.tile_nnz_at : tile_nnz_of(o); }
int32_t tile_rows_at_of(const mipdhg_options& o) { return o.tile_rows_at > 0 ? o.tile_rows_at : tile_rows_of(o); }
int32_t short_row_at_of(const mipdhg_options& o) { return o.short_row_at != 0 ? o.short_row_at : short_row_of(o); }
// What a resumed solve must share with the solve whose state it continues:
// the problem's sizes and every option that shapes the state or its layout.
uint64_t state_fingerprint(const mipdhg_lp& lp, const mipdhg_options& o) {
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the fields
    auto mix = [&](const void* p, size_t nb) {
        const unsigned char* c = (const unsigned char*)p;
        for (size_t i = 0; i < nb; ++i) h = (h ^ c[i]) * 1099511628211ull;
    };
    const int64_t sz[4] = {lp.m, lp.n, lp.nnz, (has_bounds(lp) ? 1 : 0) | (has_sense(lp) ? 2 : 0)};
    mix(sz, sizeof(sz));
    const int32_t iv[21] = {o.precision, o.ruiz_iters, o.pock_chambolle, o.power_iters, o.eval_every, o.halpern,
                            o.restarts, iter_kind(o, lp.m, lp.n), tile_nnz_of(o), tile_rows_of(o), short_row_of(o),
                            o.gather_order, o.lanes_a, o.lanes_at, o.long_row, tile_nnz_at_of(o),
                            tile_rows_at_of(o), short_row_at_of(o), o.restart_avg, o.panel_width, o.step_rule};
    mix(iv, sizeof(iv));
    const double dv[9] = {o.step_safety, o.reflect_rho, o.beta_suff, o.beta_nec, o.beta_art, o.pw_theta, o.pw_ki,
                          o.pw_kd, o.step0};
    mix(dv, sizeof(dv));
    return h;
}

// The iteration's SpMV kind.  (Every 32-bit offset of the tile kernels is
// tile-relative, so no matrix or vector size forces another kind.)
int iter_kind(const mipdhg_options& o, int64_t, int64_t) { return o.spmv_kind; }
bool sorted_layout(const mipdhg_options& o, int64_t m, int64_t n) {
    return o.gather_order == 0 && iter_kind(o, m, n) != 1;
}

TilePlan make_tile_plan(const int32_t* rowptr, const int32_t* desc, int32_t ntiles, int32_t nrows, int32_t tnz,
                        int32_t trows, int32_t srow) {
    TilePlan p;
    p.rowptr = rowptr;
    p.desc = (const int4*)desc;
    p.ntiles = ntiles;
    p.nrows = nrows;
    p.tile_nnz = tnz;
    p.tile_rows = trows;
    p.short_row = srow;
    p.max_long = srow < 0 ? 1 : tnz / (srow + 1) + 1;
    p.slot = nullptr;
    return p;
}

// Workspace layout (identical for the size query and the solve).
struct PlainWs {
    Ctrl* ctrl;
    double *d_row, *d_col, *stat_r, *stat_c, *pv, *pu, *pav, *hist, *red;
    double *pp, *pd, *per, *pec, *psetup;
    int64_t gcap;  // partial slots per kernel
    void *a_vs, *at_vs;
    // iterates relative to the anchors (u = x - x0 in x, v = y - y0 in y,
    // x_bar - x0 in xbar), anchors, absolute projected points, and the
    // anchor residuals r_c (in ct) and r_b (in bt)
    void *x, *xbar, *x0, *xhat, *ct, *y, *y0, *yhat, *bt;
    int32_t *long_a, *long_at, *tiles_a, *tiles_at, *flags;
    int32_t *col_a, *col_at;    // sorted layout: column copies in tile order
    uint16_t *slot_a, *slot_at; // sorted layout: row-major position in the tile
    void *lo_t, *hi_t;          // general form: scaled bounds l / D_c, u / D_c
    double *xprev, *yprev;      // infeasibility certificates: previous evaluated point
    double *axprev, *atyprev;   // and its A x, A^T y
    void *x_avg, *y_avg;        // restart to average: the epoch's means
    // adaptive step: the other buffer of the pairs (u, v, A~ (x - x0)) that
    // attempts alternate between, A~ (x - x0) itself, and the move's sums
    void *x_alt, *y_alt, *ax, *ax_alt;
    double *ap, *ad;
    PanelLayout pl;             // spmv_kind 3, 4: A's panel layout (dual step)
    RowPanelLayout rl;          // spmv_kind 4: A^T's row-panel layout (primal step)
    size_t bytes;
};

static PlainWs carve(void* base, size_t cap, int64_t m, int64_t n, int64_t nnz, int prec, int power_iters,
                     int64_t tnz, int64_t trows, int64_t tnz_t, int64_t trows_t, bool sorted, bool bounds,
                     bool avg, bool panel, bool adapt, bool rowpanel) {
    Carver cv(base, cap);
    PlainWs w;
    const size_t vs = prec == MIPDHG_FP64 ? 8 : (prec == MIPDHG_FP32_BF16A ? 2 : 4);
    const size_t ts = (prec == MIPDHG_FP64 || prec == MIPDHG_FP32_A) ? 8 : 4;
    w.gcap = std::max<int64_t>(kMaxRowBlocks,
                               std::max(max_tiles(m, nnz, tnz, trows), max_tiles(n, nnz, tnz_t, trows_t)));
    w.ctrl = cv.take<Ctrl>(1);
    w.d_row = cv.take<double>(m);
    w.d_col = cv.take<double>(n);
    w.stat_r = cv.take<double>(m);
    w.stat_c = cv.take<double>(n);
    w.pv = cv.take<double>(n);
    w.pu = cv.take<double>(n);
    w.pav = cv.take<double>(m);
    w.hist = cv.take<double>(power_iters + 2);
    w.red = cv.take<double>(16);
    w.pp = cv.take<double>((size_t)w.gcap * 3);
    w.pd = cv.take<double>((size_t)w.gcap * 3);
    w.per = cv.take<double>((size_t)w.gcap * kEvalRowsW);
    w.pec = cv.take<double>((size_t)w.gcap * kEvalColsW);
    w.xprev = cv.take<double>(n);
    w.yprev = cv.take<double>(m);
    w.axprev = cv.take<double>(m);
    w.atyprev = cv.take<double>(n);
    w.psetup = cv.take<double>((size_t)w.gcap * 4);
    w.a_vs = cv.take<char>(nnz * vs);
    w.at_vs = cv.take<char>(nnz * vs);
    w.x = cv.take<char>(n * ts);
    w.xbar = cv.take<char>(n * ts);
    w.x0 = cv.take<char>(n * ts);
    w.xhat = cv.take<char>(n * ts);
    w.ct = cv.take<char>(n * ts);
    w.y = cv.take<char>(m * ts);
    w.y0 = cv.take<char>(m * ts);
    w.yhat = cv.take<char>(m * ts);
    w.bt = cv.take<char>(m * ts);
    w.long_a = cv.take<int32_t>(m);
    w.long_at = cv.take<int32_t>(n);
    w.tiles_a = cv.take<int32_t>(4 * max_tiles(m, nnz, tnz, trows));
    w.tiles_at = cv.take<int32_t>(4 * max_tiles(n, nnz, tnz_t, trows_t));
    w.flags = cv.take<int32_t>(64);
    w.col_a = sorted ? cv.take<int32_t>(nnz) : nullptr;
    w.col_at = sorted ? cv.take<int32_t>(nnz) : nullptr;
    w.slot_a = sorted ? cv.take<uint16_t>(nnz) : nullptr;
    w.slot_at = sorted ? cv.take<uint16_t>(nnz) : nullptr;
    w.lo_t = bounds ? cv.take<char>(n * ts) : nullptr;
    w.hi_t = bounds ? cv.take<char>(n * ts) : nullptr;
    w.x_avg = avg ? cv.take<char>(n * ts) : nullptr;
    w.y_avg = avg ? cv.take<char>(m * ts) : nullptr;
    w.x_alt = adapt ? cv.take<char>(n * ts) : nullptr;
    w.y_alt = adapt ? cv.take<char>(m * ts) : nullptr;
    w.ax = adapt ? cv.take<char>(m * ts) : nullptr;
    w.ax_alt = adapt ? cv.take<char>(m * ts) : nullptr;
    w.ap = adapt ? cv.take<double>((size_t)w.gcap) : nullptr;
    w.ad = adapt ? cv.take<double>((size_t)w.gcap * 2) : nullptr;
    memset(&w.pl, 0, sizeof(w.pl));
    if (panel) {
        const int64_t sc = panel_seg_cap(m, nnz), cc = panel_chunk_cap(nnz), ec = panel_elem_cap(nnz);
        w.pl.groups = cv.take<PanelGroup>(kPanelMaxUnits);
        w.pl.units = cv.take<PanelUnit>(kPanelMaxUnits);
        w.pl.chunks = cv.take<PanelChunk>(cc);
        w.pl.row_group = cv.take<int32_t>(m);
        w.pl.wide_rows = cv.take<int32_t>(m);
        w.pl.counts = cv.take<int32_t>(sc);
        w.pl.seg_off = cv.take<int32_t>(sc);
        w.pl.seg_rid = cv.take<uint16_t>(sc);
        w.pl.val = cv.take<char>(ec * vs);
        w.pl.col = cv.take<uint16_t>(ec);
        w.pl.rid = cv.take<uint16_t>(ec);
        w.pl.partial = cv.take<char>(sc * ts);
    }
    memset(&w.rl, 0, sizeof(w.rl));
    if (rowpanel) {  // rows of A^T: n
        const int64_t cc = rowpanel_chunk_cap(n, nnz), ec = rowpanel_elem_cap(n, nnz);
        w.rl.groups = cv.take<RowPanelGroup>(kRowPanelMaxUnits);
        w.rl.units = cv.take<RowPanelUnit>(kRowPanelMaxUnits);
        w.rl.chunks = cv.take<PanelChunk>(cc);
        w.rl.val = cv.take<char>(ec * vs);
        w.rl.col = cv.take<uint16_t>(ec);
        w.rl.rid = cv.take<uint16_t>(ec);
        w.rl.row_group = cv.take<int32_t>(n);
        w.rl.row_off = cv.take<int32_t>(n);
        w.rl.row_rid = cv.take<uint16_t>(n);
        w.rl.span = cv.take<int32_t>(2 * std::max(m, n));
    }
    w.bytes = (cv.off + 255) & ~size_t(255);
    return w;
}

int check_options(const mipdhg_options* o) {
    if (o->precision < 0 || o->precision > 4) return set_error("precision must be 0 to 4"), MIPDHG_ERR_INVALID_ARG;
    if (o->ruiz_iters < 0 || o->power_iters < 1 || o->power_iters > 100000)
        return set_error("ruiz_iters >= 0 and 1 <= power_iters <= 100000 required"), MIPDHG_ERR_INVALID_ARG;
    if (o->eval_every < 1 || o->eval_every > 4096)
        return set_error("eval_every must be in [1, 4096]"), MIPDHG_ERR_INVALID_ARG;
    if (!(o->step_safety > 0.0) || !(o->reflect_rho >= 0.0 && o->reflect_rho <= 1.0))
        return set_error("step_safety > 0 and reflect_rho in [0,1] required"), MIPDHG_ERR_INVALID_ARG;
    if (o->max_iter < 1) return set_error("max_iter must be >= 1"), MIPDHG_ERR_INVALID_ARG;
    if (!(o->pw_theta >= 0.0 && o->pw_theta <= 1.0)) return set_error("pw_theta must be in [0,1]"), MIPDHG_ERR_INVALID_ARG;
    if (!std::isfinite(o->pw_ki) || !std::isfinite(o->pw_kd))
        return set_error("pw_ki and pw_kd must be finite"), MIPDHG_ERR_INVALID_ARG;
    if (o->spmv_kind < 0 || o->spmv_kind > 4) return set_error("spmv_kind must be 0 to 4"), MIPDHG_ERR_INVALID_ARG;
    if (o->panel_width != 0) {
        const int maxw = kPanelBytes / ((o->precision == MIPDHG_FP64 || o->precision == MIPDHG_FP32_A) ? 8 : 4);
        if (o->panel_width < 64 || o->panel_width > maxw || (o->panel_width & (o->panel_width - 1)))
            return set_error("panel_width must be 0 or a power of two in [64, %d]", maxw), MIPDHG_ERR_INVALID_ARG;
    }
    if (o->gather_order < 0 || o->gather_order > 1) return set_error("gather_order must be 0 or 1"), MIPDHG_ERR_INVALID_ARG;
    if (o->kernel_timing < 0 || o->kernel_timing > 2)
        return set_error("kernel_timing must be 0, 1 or 2"), MIPDHG_ERR_INVALID_ARG;
    if (o->resume < 0 || o->resume > 1) return set_error("resume must be 0 or 1"), MIPDHG_ERR_INVALID_ARG;
    if (!(o->infeas_tol >= 0.0) || !std::isfinite(o->infeas_tol))
        return set_error("infeas_tol must be finite and >= 0"), MIPDHG_ERR_INVALID_ARG;
    if (o->resume && (o->x_init || o->y_init || o->trace_iters))
        return set_error("resume continues the workspace's state: no warm start or trace with it"),
               MIPDHG_ERR_INVALID_ARG;
    if (o->tile_nnz != 0 && (o->tile_nnz < 256 || o->tile_nnz > kMaxTileNnz))
        return set_error("tile_nnz must be 0 or in [256, %d]", kMaxTileNnz), MIPDHG_ERR_INVALID_ARG;
    if (o->tile_rows < 0 || o->tile_rows > kMaxTileRows)
        return set_error("tile_rows must be in [0, %d]", kMaxTileRows), MIPDHG_ERR_INVALID_ARG;
    if (o->short_row < -1) return set_error("short_row must be >= -1"), MIPDHG_ERR_INVALID_ARG;
    if (o->tile_nnz_at != 0 && (o->tile_nnz_at < 256 || o->tile_nnz_at > kMaxTileNnz))
        return set_error("tile_nnz_at must be 0 or in [256, %d]", kMaxTileNnz), MIPDHG_ERR_INVALID_ARG;
    if (o->tile_rows_at < 0 || o->tile_rows_at > kMaxTileRows)
        return set_error("tile_rows_at must be in [0, %d]", kMaxTileRows), MIPDHG_ERR_INVALID_ARG;
    if (o->short_row_at < -1) return set_error("short_row_at must be >= -1"), MIPDHG_ERR_INVALID_ARG;
    if (o->restart_avg < 0 || o->restart_avg > 1) return set_error("restart_avg must be 0 or 1"), MIPDHG_ERR_INVALID_ARG;
    if (o->batch_split < 0 || o->batch_split > 150 * 1024)
        return set_error("batch_split must be in [0, 153600] bytes"), MIPDHG_ERR_INVALID_ARG;
    if (o->batch_block_iters < 0) return set_error("batch_block_iters must be >= 0"), MIPDHG_ERR_INVALID_ARG;
    if (o->step_rule < 0 || o->step_rule > 1) return set_error("step_rule must be 0 or 1"), MIPDHG_ERR_INVALID_ARG;
    if (!(o->step0 >= 0.0) || !std::isfinite(o->step0))
        return set_error("step0 must be finite and >= 0"), MIPDHG_ERR_INVALID_ARG;
    if (o->step_rule == 1 && (o->halpern != 0 || o->reflect_rho != 0.0 || o->restart_avg != 0))
        return set_error("step_rule 1 needs plain PDHG: halpern 0, reflect_rho 0, restart_avg 0"),
               MIPDHG_ERR_INVALID_ARG;
    for (int L : {o->lanes_a, o->lanes_at})
        if (L != 0 && L != 2 && L != 4 && L != 8 && L != 16 && L != 32 && L != 64)
            return set_error("lanes must be 0 or a power of two in [2, 64]"), MIPDHG_ERR_INVALID_ARG;
    if (o->trace_iters < 0) return set_error("trace_iters must be >= 0"), MIPDHG_ERR_INVALID_ARG;
    return 0;
}

int check_lp(const mipdhg_lp* lp) {
    if (!lp) return set_error("lp is NULL"), MIPDHG_ERR_INVALID_ARG;
    if (lp->m < 1 || lp->n < 1 || lp->nnz < 0 || lp->nnz >= (int64_t)INT32_MAX)
        return set_error("need m >= 1, n >= 1 and 0 <= nnz < 2^31 (m=%d n=%d nnz=%lld)", lp->m, lp->n,
                         (long long)lp->nnz),
               MIPDHG_ERR_INVALID_ARG;
    if (!lp->a_rowptr || !lp->at_rowptr || !lp->b || !lp->c ||
        (lp->nnz > 0 && (!lp->a_col || !lp->a_val || !lp->at_col || !lp->at_val)))
        return set_error("a required LP pointer is NULL"), MIPDHG_ERR_INVALID_ARG;
    return 0;
}

int check_rowptr(const std::vector<int32_t>& rp, int32_t nrows, int64_t nnz, const char* which) {
    if (rp[0] != 0 || (int64_t)rp[nrows] != nnz)
        return set_error("%s row pointer must start at 0 and end at nnz", which), MIPDHG_ERR_BAD_CSR;
    for (int32_t r = 0; r < nrows; ++r)
        if (rp[r + 1] < rp[r]) return set_error("%s row pointer decreases at row %d", which, r), MIPDHG_ERR_BAD_CSR;
    return 0;
}

}  // namespace mip

using namespace mip;

extern "C" int mipdhg_workspace_size(const mipdhg_lp* lp, const mipdhg_options* opt, size_t* bytes) {
    clear_error();
    if (!bytes || !opt) return set_error("NULL argument"), MIPDHG_ERR_INVALID_ARG;
    int rc = check_lp(lp);
    if (rc) return rc;
    if ((rc = check_options(opt))) return rc;
    *bytes = carve(nullptr, 0, lp->m, lp->n, lp->nnz, opt->precision, opt->power_iters, tile_nnz_of(*opt),
                   tile_rows_of(*opt), tile_nnz_at_of(*opt), tile_rows_at_of(*opt), sorted_layout(*opt, lp->m, lp->n),
                   has_bounds(*lp), opt->restart_avg != 0, opt->spmv_kind >= 3, opt->step_rule == 1, opt->spmv_kind == 4).bytes;
    return 0;
}

namespace mip {

template <typename T, typename V, typename Acc>
struct Solver {
    const mipdhg_lp& lp;
    const mipdhg_options& o;
    hipStream_t stream;
    PlainWs w;
    HostPlan hpa, hpat;   // lane-group plans (spmv_kind 1, transpose test)
    RowPlan pa, pat;
    TilePlan ta, tat;     // LDS tile plans
    double *xo, *yo, *zo, *rpo, *rdo;
    // kernel timing: three events per iteration (before primal, between, after dual)
    bool timing = false;
    std::vector<hipEvent_t> tev;
    double ms_p = 0.0, ms_d = 0.0;
    int64_t n_p = 0, n_d = 0;

    Solver(const mipdhg_lp& l, const mipdhg_options& op, hipStream_t s) : lp(l), o(op), stream(s) {}
    ~Solver() {
        for (auto e : tev)
            if (e) (void)hipEventDestroy(e);
    }
    bool tiled() const { return iter_kind(o, lp.m, lp.n) != 1; }
    bool persistent() const { return iter_kind(o, lp.m, lp.n) == 2; }
    int gp_persist = 0, gd_persist = 0;  // persistent grids (resident slots, capped by the tile count)
    // dynamic LDS beyond 64 KiB must be allowed per kernel
    int allow_tile_lds() {
        const size_t need = std::max(tile_lds_bytes(ta, 8), tile_lds_bytes(tat, 8));
        if (need > 65536) {
            const int lim = (int)need;
#define MIP_ITER_KERNELS(G)                                                                                  \
    (const void*)k_iter_tiled<T, V, Acc, true, 8, false, G>, (const void*)k_iter_tiled<T, V, Acc, false, 8, false, G>,  \
        (const void*)k_iter_tiled<T, V, Acc, true, 16, false, G>,                                                      \
        (const void*)k_iter_tiled<T, V, Acc, false, 16, false, G>, (const void*)k_iter_tiled<T, V, Acc, true, 8, true, G>, \
        (const void*)k_iter_tiled<T, V, Acc, false, 8, true, G>, (const void*)k_iter_tiled<T, V, Acc, true, 16, true, G>, \
        (const void*)k_iter_tiled<T, V, Acc, false, 16, true, G>, (const void*)k_iter_persist<T, V, Acc, true, 8, false, G>, \
        (const void*)k_iter_persist<T, V, Acc, false, 8, false, G>,                                                    \
        (const void*)k_iter_persist<T, V, Acc, true, 16, false, G>,                                                    \
        (const void*)k_iter_persist<T, V, Acc, false, 16, false, G>,                                                   \
        (const void*)k_iter_persist<T, V, Acc, true, 8, true, G>, (const void*)k_iter_persist<T, V, Acc, false, 8, true, G>, \
        (const void*)k_iter_persist<T, V, Acc, true, 16, true, G>,                                                     \
        (const void*)k_iter_persist<T, V, Acc, false, 16, true, G>
#define MIP_AVG_KERNELS(G)                                                                                   \
    (const void*)k_iter_tiled<T, V, Acc, true, 8, false, G, true>,                                            \
        (const void*)k_iter_tiled<T, V, Acc, false, 8, false, G, true>,                                       \
        (const void*)k_iter_tiled<T, V, Acc, true, 16, false, G, true>,                                       \
        (const void*)k_iter_tiled<T, V, Acc, false, 16, false, G, true>,                                      \
        (const void*)k_iter_tiled<T, V, Acc, true, 8, true, G, true>,                                         \
        (const void*)k_iter_tiled<T, V, Acc, false, 8, true, G, true>,                                        \
        (const void*)k_iter_tiled<T, V, Acc, true, 16, true, G, true>,                                        \
        (const void*)k_iter_tiled<T, V, Acc, false, 16, true, G, true>
#define MIP_ADAPT_KERNELS(G)                                                                                 \
    (const void*)k_iter_tiled<T, V, Acc, true, 8, false, G, false, true>,                                     \
        (const void*)k_iter_tiled<T, V, Acc, false, 8, false, G, false, true>,                                \
        (const void*)k_iter_tiled<T, V, Acc, true, 16, false, G, false, true>,                                \
        (const void*)k_iter_tiled<T, V, Acc, false, 16, false, G, false, true>,                               \
        (const void*)k_iter_tiled<T, V, Acc, true, 8, true, G, false, true>,                                  \
        (const void*)k_iter_tiled<T, V, Acc, false, 8, true, G, false, true>,                                 \
        (const void*)k_iter_tiled<T, V, Acc, true, 16, true, G, false, true>,                                 \
        (const void*)k_iter_tiled<T, V, Acc, false, 16, true, G, false, true>
            const void* ks[] = {MIP_ITER_KERNELS(false), MIP_ITER_KERNELS(true), MIP_AVG_KERNELS(false),
                                MIP_AVG_KERNELS(true), MIP_ADAPT_KERNELS(false), MIP_ADAPT_KERNELS(true),
                                (const void*)k_eval<true, false>, (const void*)k_eval<false, false>,
                                (const void*)k_eval<true, true>, (const void*)k_eval<false, true>,
                                (const void*)k_scale_stat<true>, (const void*)k_scale_stat<false>,
                                (const void*)k_anchor_resid<T>,
                                (const void*)k_spmv_copy<V, true, T, 8>, (const void*)k_spmv_copy<V, false, T, 8>,
                                (const void*)k_spmv_copy<V, true, T, 16>, (const void*)k_spmv_copy<V, false, T, 16>};
#undef MIP_ITER_KERNELS
#undef MIP_AVG_KERNELS
#undef MIP_ADAPT_KERNELS
            for (const void* k : ks)
                if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess)
                    return set_error("tile shape needs %d bytes of LDS per workgroup, more than the device allows", lim),
                           MIPDHG_ERR_UNSUPPORTED;
            int rc = allow_validate_lds(lim);
            if (rc) return rc;
        }
        const size_t sneed = std::max(sort_lds_bytes(ta), sort_lds_bytes(tat));
        if (sorted() && sneed > 65536 &&
            hipFuncSetAttribute((const void*)k_sort_scale_tiles<V>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sneed) != hipSuccess)
            return set_error("tile sort needs %zu bytes of LDS per workgroup, more than the device allows", sneed),
                   MIPDHG_ERR_UNSUPPORTED;
        return 0;
    }
    bool sorted() const { return sorted_layout(o, lp.m, lp.n); }
    // spmv_kind 3: the dual step on A's panel layout, the primal on A^T's tiles
    bool panel() const { return o.spmv_kind == 3 || o.spmv_kind == 4; }
    bool rowpanel() const { return o.spmv_kind == 4; }
    int panel_w() const { return o.panel_width > 0 ? o.panel_width : panel_width<T>(); }
    int grid_primal() const {
        if (rowpanel()) return w.rl.nunits;
        return persistent() ? gp_persist : tiled() ? tat.ntiles : hpat.grid();
    }
    int grid_dual() const {
        if (panel())
            return (int)((lp.m + kBlock - 1) / kBlock + (w.pl.nwide + kBlock / kWave - 1) / (kBlock / kWave));
        return persistent() ? gd_persist : tiled() ? ta.ntiles : hpa.grid();
    }
    // Resident workgroups of the persistent kernel over all CUs, at least
    // min(8, ntiles) so that every XCD's run of tiles has a workgroup.
    // the general-form variant of a kernel: bounds for the primal, senses for the dual
    bool gen_primal() const { return has_bounds(lp); }
    bool gen_dual() const { return has_sense(lp); }
    template <bool PRIMAL>
    int persist_grid(const TilePlan& tp) {
        return (PRIMAL ? gen_primal() : gen_dual()) ? persist_grid_g<PRIMAL, true>(tp) : persist_grid_g<PRIMAL, false>(tp);
    }
    template <bool PRIMAL, bool G>
    int persist_grid_g(const TilePlan& tp) {
        int dev = 0, cus = 0, occ = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        const size_t lds = tile_lds_bytes(tp, sizeof(Acc));
        hipError_t e;
        if (tp.tile_nnz > 8 * kBlock)
            e = sorted() ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                               &occ, k_iter_persist<T, V, Acc, PRIMAL, 16, true, G>, kBlock, lds)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                               &occ, k_iter_persist<T, V, Acc, PRIMAL, 16, false, G>, kBlock, lds);
        else
            e = sorted() ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                               &occ, k_iter_persist<T, V, Acc, PRIMAL, 8, true, G>, kBlock, lds)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                               &occ, k_iter_persist<T, V, Acc, PRIMAL, 8, false, G>, kBlock, lds);
        if (e != hipSuccess || occ < 1) return 0;
        const int64_t g = std::min<int64_t>((int64_t)cus * occ, tp.ntiles);
        return (int)std::max<int64_t>(g, std::min<int64_t>(8, tp.ntiles));
    }
    int plan_persistent() {
        if (!persistent()) return 0;
        gp_persist = persist_grid<true>(tat);
        gd_persist = persist_grid<false>(ta);
        if (gp_persist < 1 || gd_persist < 1)
            return set_error("could not size the persistent grid (occupancy query failed)"), MIPDHG_ERR_HIP;
        return 0;
    }

    void fill_iter(IterArgs<T, V>& a, bool primal, int it, int flags) {
        a.p = primal ? pat : pa;
        a.col = primal ? (sorted() ? w.col_at : lp.at_col) : (sorted() ? w.col_a : lp.a_col);
        a.val = (const V*)(primal ? w.at_vs : w.a_vs);
        a.gather = (const T*)(primal ? w.y : w.xbar);
        a.state = (T*)(primal ? w.x : w.y);
        a.bar = primal ? (T*)w.xbar : nullptr;
        a.hat = (T*)(primal ? w.xhat : w.yhat);
        a.anchor = (const T*)(primal ? w.x0 : w.y0);
        a.rhs = (const T*)(primal ? w.ct : w.bt);
        a.out64 = primal ? xo : yo;
        a.dscale = primal ? w.d_col : w.d_row;
        a.partials = primal ? w.pp : w.pd;
        a.ctrl = w.ctrl;
        a.lo = (const T*)w.lo_t;
        a.hi = (const T*)w.hi_t;
        a.sense = lp.sense;
        a.avg = (T*)(primal ? w.x_avg : w.y_avg);
        a.rho = o.reflect_rho;
        a.halpern = o.halpern;
        a.it = it;
        a.flags = flags;
        a.state_out = a.state;
        a.ax_in = nullptr;
        a.ax_out = nullptr;
        a.apart = nullptr;
        if (adaptive()) {  // even attempts go from the first buffers to the second, odd ones back
            const bool odd = (it & 1) != 0;
            void* const xin = odd ? w.x_alt : w.x;
            void* const xout = odd ? w.x : w.x_alt;
            void* const yin = odd ? w.y_alt : w.y;
            void* const yout = odd ? w.y : w.y_alt;
            a.state = (T*)(primal ? xin : yin);
            a.state_out = (T*)(primal ? xout : yout);
            if (primal) a.gather = (const T*)yin;
            a.ax_in = (const T*)(odd ? w.ax_alt : w.ax);
            a.ax_out = (T*)(odd ? w.ax : w.ax_alt);
            a.apart = primal ? w.ap : w.ad;
        }
    }
    bool adaptive() const { return o.step_rule == 1; }
    // One of the tile kernels: one workgroup per tile or persistent, 8 or 16
    // products in flight per thread, row-major or sorted layout.
    template <bool PRIMAL>
    void launch_tiles(const IterArgs<T, V>& a, TilePlan tp, int gpersist) {
        const bool g = PRIMAL ? gen_primal() : gen_dual();
        if (o.restart_avg) {  // one workgroup per tile only (checked with the options)
            if (g) launch_tiles_g<PRIMAL, true, true>(a, tp, gpersist);
            else launch_tiles_g<PRIMAL, false, true>(a, tp, gpersist);
        } else if (adaptive()) {  // likewise
            if (g) launch_tiles_g<PRIMAL, true, false, true>(a, tp, gpersist);
            else launch_tiles_g<PRIMAL, false, false, true>(a, tp, gpersist);
        } else {
            if (g) launch_tiles_g<PRIMAL, true, false>(a, tp, gpersist);
            else launch_tiles_g<PRIMAL, false, false>(a, tp, gpersist);
        }
    }
    template <bool PRIMAL, bool G, bool AVG, bool ADAPT = false>
    void launch_tiles_g(const IterArgs<T, V>& a, TilePlan tp, int gpersist) {
        const size_t lds = tile_lds_bytes(tp, sizeof(Acc));
        const bool big = tp.tile_nnz > 8 * kBlock;
        const dim3 grid(persistent() ? gpersist : tp.ntiles);
        if (sorted()) tp.slot = PRIMAL ? w.slot_at : w.slot_a;
#define MIP_TILE_LAUNCH(K, U, SRT) \
    hipLaunchKernelGGL((K<T, V, Acc, PRIMAL, U, SRT, G>), grid, dim3(kBlock), lds, stream, a, tp)
#define MIP_AVG_LAUNCH(U, SRT) \
    hipLaunchKernelGGL((k_iter_tiled<T, V, Acc, PRIMAL, U, SRT, G, true>), grid, dim3(kBlock), lds, stream, a, tp)
#define MIP_ADAPT_LAUNCH(U, SRT)                                                                              \
    hipLaunchKernelGGL((k_iter_tiled<T, V, Acc, PRIMAL, U, SRT, G, false, true>), grid, dim3(kBlock), lds, stream, \
                       a, tp)
        if constexpr (ADAPT) {
            if (big) {
                if (sorted()) MIP_ADAPT_LAUNCH(16, true);
                else MIP_ADAPT_LAUNCH(16, false);
            } else {
                if (sorted()) MIP_ADAPT_LAUNCH(8, true);
                else MIP_ADAPT_LAUNCH(8, false);
            }
        } else if constexpr (AVG) {
            if (big) {
                if (sorted()) MIP_AVG_LAUNCH(16, true);
                else MIP_AVG_LAUNCH(16, false);
            } else {
                if (sorted()) MIP_AVG_LAUNCH(8, true);
                else MIP_AVG_LAUNCH(8, false);
            }
        } else if (persistent()) {
            if (big) {
                if (sorted()) MIP_TILE_LAUNCH(k_iter_persist, 16, true);
                else MIP_TILE_LAUNCH(k_iter_persist, 16, false);
            } else {
                if (sorted()) MIP_TILE_LAUNCH(k_iter_persist, 8, true);
                else MIP_TILE_LAUNCH(k_iter_persist, 8, false);
            }
        } else {
            if (big) {
                if (sorted()) MIP_TILE_LAUNCH(k_iter_tiled, 16, true);
                else MIP_TILE_LAUNCH(k_iter_tiled, 16, false);
            } else {
                if (sorted()) MIP_TILE_LAUNCH(k_iter_tiled, 8, true);
                else MIP_TILE_LAUNCH(k_iter_tiled, 8, false);
            }
        }
#undef MIP_TILE_LAUNCH
#undef MIP_AVG_LAUNCH
#undef MIP_ADAPT_LAUNCH
    }
    int launch_primal(int it, int flags) {
        IterArgs<T, V> a;
        fill_iter(a, true, it, flags);
        if (rowpanel()) {
            RowPanelArgs<V> ra;
            ra.width = panel_w();
            ra.groups = w.rl.groups;
            ra.units = w.rl.units;
            ra.chunks = w.rl.chunks;
            ra.val = (const V*)w.rl.val;
            ra.col = w.rl.col;
            ra.rid = w.rl.rid;
            ra.t0 = w.rl.t0;
            ra.tail = w.rl.tail;
            ra.ncols = lp.m;
            if (w.rl.nunits > 0) {
                if (gen_primal())
                    hipLaunchKernelGGL((k_rowpanel_primal<T, V, true>), dim3(w.rl.nunits), dim3(kPanelBlock), 0,
                                       stream, a, ra);
                else
                    hipLaunchKernelGGL((k_rowpanel_primal<T, V, false>), dim3(w.rl.nunits), dim3(kPanelBlock), 0,
                                       stream, a, ra);
            }
        } else if (tiled()) {
            launch_tiles<true>(a, tat, gp_persist);
        } else {
            MIP_DISPATCH_L(pat.lanes, hipLaunchKernelGGL((k_iter<T, V, Acc, L, true>), dim3(hpat.grid()), dim3(kBlock),
                                                         0, stream, a));
        }
        MIP_LAUNCH_CHECK();
        return 0;
    }
    int launch_dual(int it, int flags) {
        IterArgs<T, V> a;
        fill_iter(a, false, it, flags);
        if (panel()) {
            PanelArgs<T, V> pa;
            pa.width = panel_w();
            pa.groups = w.pl.groups;
            pa.units = w.pl.units;
            pa.chunks = w.pl.chunks;
            pa.val = (const V*)w.pl.val;
            pa.col = w.pl.col;
            pa.rid = w.pl.rid;
            pa.gather = (const T*)w.xbar;
            pa.partial = (T*)w.pl.partial;
            pa.ncols = lp.n;
            pa.ctrl = w.ctrl;
            if (w.pl.nunits > 0)
                hipLaunchKernelGGL((k_panel_spmv<T, V>), dim3(w.pl.nunits), dim3(kPanelBlock), 0, stream, pa);
            const PanelRows pr{w.pl.groups, w.pl.row_group, w.pl.wide_rows, lp.m, w.pl.nwide};
            if (gen_dual())
                hipLaunchKernelGGL((k_panel_rows<T, V, true>), dim3(grid_dual()), dim3(kBlock), 0, stream, a, pr,
                                   (const T*)w.pl.partial);
            else
                hipLaunchKernelGGL((k_panel_rows<T, V, false>), dim3(grid_dual()), dim3(kBlock), 0, stream, a, pr,
                                   (const T*)w.pl.partial);
        } else if (tiled()) {
            launch_tiles<false>(a, ta, gd_persist);
        } else {
            MIP_DISPATCH_L(pa.lanes, hipLaunchKernelGGL((k_iter<T, V, Acc, L, false>), dim3(hpa.grid()), dim3(kBlock),
                                                        0, stream, a));
        }
        MIP_LAUNCH_CHECK();
        return 0;
    }
    int launch_eval_and_decide(int nit) {
        EvalArgs er;
        er.col = lp.a_col;
        er.val = lp.a_val;
        er.gather = xo;
        er.vec = lp.b;
        er.own = yo;
        er.out1 = rpo;
        er.out2 = nullptr;
        er.partials = w.per;
        er.ctrl = w.ctrl;
        er.sense = lp.sense;
        er.lo = er.hi = nullptr;
        er.prod_prev = w.axprev;
        er.own_prev = w.yprev;
        er.rays = o.infeas_tol > 0.0;
        if (gen_dual())
            hipLaunchKernelGGL((k_eval<true, true>), dim3(ta.ntiles), dim3(kBlock), tile_lds_bytes(ta, 8), stream, er,
                               ta);
        else
            hipLaunchKernelGGL((k_eval<true, false>), dim3(ta.ntiles), dim3(kBlock), tile_lds_bytes(ta, 8), stream,
                               er, ta);
        MIP_LAUNCH_CHECK();
        EvalArgs ec;
        ec.col = lp.at_col;
        ec.val = lp.at_val;
        ec.gather = yo;
        ec.vec = lp.c;
        ec.own = xo;
        ec.out1 = zo;
        ec.out2 = rdo;
        ec.partials = w.pec;
        ec.ctrl = w.ctrl;
        ec.sense = nullptr;
        ec.lo = lp.lo;
        ec.hi = lp.hi;
        ec.prod_prev = w.atyprev;
        ec.own_prev = w.xprev;
        ec.rays = o.infeas_tol > 0.0;
        if (gen_primal())
            hipLaunchKernelGGL((k_eval<false, true>), dim3(tat.ntiles), dim3(kBlock), tile_lds_bytes(tat, 8), stream,
                               ec, tat);
        else
            hipLaunchKernelGGL((k_eval<false, false>), dim3(tat.ntiles), dim3(kBlock), tile_lds_bytes(tat, 8),
                               stream, ec, tat);
        MIP_LAUNCH_CHECK();
        return launch_decide(nit);
    }
    // decision and restart copy for a block of nit iterations whose
    // evaluation partials are in the workspace
    int launch_decide(int nit) {
        DecideArgs d;
        d.ctrl = w.ctrl;
        d.pp = w.pp;
        d.pd = w.pd;
        d.per = w.per;
        d.pec = w.pec;
        d.gp = grid_primal();
        d.gd = grid_dual();
        d.ger = ta.ntiles;
        d.gec = tat.ntiles;
        d.nit = nit;
        hipLaunchKernelGGL(k_decide, dim3(1), dim3(kBlock), 0, stream, d);
        MIP_LAUNCH_CHECK();
        const int64_t mx = std::max<int64_t>(lp.m, lp.n);
        // the restart point: the evaluation's projected point, or the epoch average
        const T* rx = (const T*)(o.restart_avg ? w.x_avg : w.xhat);
        const T* ry = (const T*)(o.restart_avg ? w.y_avg : w.yhat);
        hipLaunchKernelGGL((k_apply_restart<T>), dim3(grid_for(mx)), dim3(kBlock), 0, stream,
                           (const Ctrl*)w.ctrl, (T*)w.x, (T*)w.x0, rx, (int64_t)lp.n, (T*)w.y, (T*)w.y0, ry,
                           (int64_t)lp.m, (T*)w.ax);
        MIP_LAUNCH_CHECK();
        return launch_anchor_resid(0);
    }
    // r_b, r_c of the current anchor (force: whatever the restart flag says)
    // (the power iteration's vectors, free after setup, hold D_c x0 and D_r y0)
    int launch_anchor_resid(int force) {
        const Ctrl* c = (const Ctrl*)w.ctrl;
        hipLaunchKernelGGL((k_anchor_scale<T>), dim3(grid_for(lp.n)), dim3(kBlock), 0, stream,
                           (const double*)w.d_col, (const T*)w.x0, (int64_t)lp.n, w.pu, c, force);
        hipLaunchKernelGGL((k_anchor_scale<T>), dim3(grid_for(lp.m)), dim3(kBlock), 0, stream,
                           (const double*)w.d_row, (const T*)w.y0, (int64_t)lp.m, w.pav, c, force);
        hipLaunchKernelGGL((k_anchor_resid<T>), dim3(ta.ntiles), dim3(kBlock), tile_lds_bytes(ta, 8), stream, ta,
                           lp.a_col, lp.a_val, (const double*)w.d_row, (const double*)w.pu, lp.b, (T*)w.bt, c,
                           force);
        hipLaunchKernelGGL((k_anchor_resid<T>), dim3(tat.ntiles), dim3(kBlock), tile_lds_bytes(tat, 8), stream, tat,
                           lp.at_col, lp.at_val, (const double*)w.d_col, (const double*)w.pav, lp.c, (T*)w.ct, c,
                           force);
        MIP_LAUNCH_CHECK();
        return 0;
    }
    // The adaptive step's decision on attempt it, and the rollback of a
    // rejected attempt
    int launch_step(int it, int flags) {
        StepArgs sa{w.ctrl, w.ap, w.ad, grid_primal(), grid_dual(), it};
        hipLaunchKernelGGL(k_step, dim3(1), dim3(kBlock), 0, stream, sa);
        const bool odd = (it & 1) != 0;
        RestoreArgs<T> ra;
        ra.ctrl = w.ctrl;
        ra.u_in = (const T*)(odd ? w.x_alt : w.x);
        ra.u_out = (T*)(odd ? w.x : w.x_alt);
        ra.v_in = (const T*)(odd ? w.y_alt : w.y);
        ra.v_out = (T*)(odd ? w.y : w.y_alt);
        ra.ax_in = (const T*)(odd ? w.ax_alt : w.ax);
        ra.ax_out = (T*)(odd ? w.ax : w.ax_alt);
        ra.x0 = (const T*)w.x0;
        ra.y0 = (const T*)w.y0;
        ra.xhat = (T*)w.xhat;
        ra.yhat = (T*)w.yhat;
        ra.xo = xo;
        ra.yo = yo;
        ra.d_col = w.d_col;
        ra.d_row = w.d_row;
        ra.pp = w.pp;
        ra.pd = w.pd;
        ra.n = lp.n;
        ra.m = lp.m;
        ra.gp = grid_primal();
        ra.gd = grid_dual();
        ra.flags = flags;
        hipLaunchKernelGGL((k_adapt_restore<T>), dim3(std::max(ra.gp, ra.gd)), dim3(kBlock), 0, stream, ra);
        MIP_LAUNCH_CHECK();
        return 0;
    }
    // One block of nit iterations ending in an evaluation.  With trace, the
    // scaled iterates after iteration t_first + i are exported.
    int enqueue_block(int nit, int64_t t_first, bool trace) {
        int rc;
        for (int it = 0; it < nit; ++it) {
            const bool last = it == nit - 1;
            const int flags = (it == 0 ? F_FIRST : 0) | (last ? (F_EVAL | F_HAT) : 0) | (trace ? F_HAT : 0);
            if (timing) MIP_HIP(hipEventRecord(tev[3 * it], stream));
            if ((rc = launch_primal(it, flags))) return rc;
            if (timing) MIP_HIP(hipEventRecord(tev[3 * it + 1], stream));
            if ((rc = launch_dual(it, flags))) return rc;
            if (timing) MIP_HIP(hipEventRecord(tev[3 * it + 2], stream));
            if (adaptive()) {
                if ((rc = launch_step(it, flags))) return rc;
                if (last && (nit & 1)) {  // an odd block ends in the second buffers
                    hipLaunchKernelGGL((k_copy_iterate<T>), dim3(grid_for(std::max(lp.m, lp.n))), dim3(kBlock), 0,
                                       stream, (const T*)w.x_alt, (T*)w.x, (int64_t)lp.n, (const T*)w.y_alt, (T*)w.y,
                                       (const T*)w.ax_alt, (T*)w.ax, (int64_t)lp.m);
                    MIP_LAUNCH_CHECK();
                }
            }
            if (last && (rc = launch_eval_and_decide(nit))) return rc;
            const int64_t t = t_first + it;  // 1-based iteration number
            if (trace && t <= o.trace_iters) {
                const int64_t off_n = (t - 1) * (int64_t)lp.n, off_m = (t - 1) * (int64_t)lp.m;
                // the adaptive step's even attempts (but a block's last) leave the iterate in the second buffers
                const bool second = adaptive() && !last && (it & 1) == 0;
                if (o.trace_x)
                    hipLaunchKernelGGL((k_export<T>), dim3(grid_for(lp.n)), dim3(kBlock), 0, stream,
                                       (const T*)(second ? w.x_alt : w.x), (const T*)w.x0, o.trace_x + off_n,
                                       (int64_t)lp.n);
                if (o.trace_y)
                    hipLaunchKernelGGL((k_export<T>), dim3(grid_for(lp.m)), dim3(kBlock), 0, stream,
                                       (const T*)(second ? w.y_alt : w.y), (const T*)w.y0, o.trace_y + off_m,
                                       (int64_t)lp.m);
                if (o.trace_xhat)
                    hipLaunchKernelGGL((k_export<T>), dim3(grid_for(lp.n)), dim3(kBlock), 0, stream,
                                       (const T*)w.xhat, (const T*)nullptr, o.trace_xhat + off_n, (int64_t)lp.n);
                if (o.trace_yhat)
                    hipLaunchKernelGGL((k_export<T>), dim3(grid_for(lp.m)), dim3(kBlock), 0, stream,
                                       (const T*)w.yhat, (const T*)nullptr, o.trace_yhat + off_m, (int64_t)lp.m);
                MIP_LAUNCH_CHECK();
            }
        }
        if (timing) {
            MIP_HIP(hipEventSynchronize(tev[3 * (nit - 1) + 2]));
            for (int it = 0; it < nit; ++it) {
                float a = 0.f, b = 0.f;
                MIP_HIP(hipEventElapsedTime(&a, tev[3 * it], tev[3 * it + 1]));
                MIP_HIP(hipEventElapsedTime(&b, tev[3 * it + 1], tev[3 * it + 2]));
                ms_p += a;
                ms_d += b;
            }
            n_p += nit;
            n_d += nit;
        }
        return 0;
    }
};

template <typename T, typename V, typename Acc>
static int solve_impl(const mipdhg_lp& lp, const mipdhg_options& o, double eps, void* ws, size_t ws_bytes,
                      hipStream_t stream, double* x, double* y, double* z, double* r_p, double* r_d,
                      double* d_row, double* d_col, mipdhg_info* info) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    Solver<T, V, Acc> S(lp, o, stream);
    S.w = carve(ws, ws_bytes, lp.m, lp.n, lp.nnz, o.precision, o.power_iters, tile_nnz_of(o), tile_rows_of(o),
                tile_nnz_at_of(o), tile_rows_at_of(o), sorted_layout(o, lp.m, lp.n), has_bounds(lp),
                o.restart_avg != 0, o.spmv_kind >= 3, o.step_rule == 1, o.spmv_kind == 4);
    if (S.w.bytes > ws_bytes)
        return set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, S.w.bytes),
               MIPDHG_ERR_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return set_error("workspace must be 256-byte aligned"), MIPDHG_ERR_INVALID_ARG;
    S.xo = x;
    S.yo = y;
    S.zo = z;
    S.rpo = r_p;
    S.rdo = r_d;
    PlainWs& w = S.w;
    const int64_t m = lp.m, n = lp.n, nnz = lp.nnz;
    // a resumed solve checks the state's sizes and options before setup
    // writes to the workspace (the control block is at its start whatever
    // the layout), so that a refused resume leaves the state as it was
    const uint64_t fp = state_fingerprint(lp, o);
    if (o.resume) {
        Ctrl cur;
        MIP_HIP(hipMemcpyAsync(&cur, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
        MIP_HIP(hipStreamSynchronize(stream));
        if (!cur.resumable || cur.fingerprint != fp)
            return set_error("resume: the workspace does not hold a resumable state of this LP with these options"),
                   MIPDHG_ERR_INVALID_ARG;
        if (cur.status == MIPDHG_NUMERICAL)
            return set_error("resume: the stopped solve hit non-finite values"), MIPDHG_ERR_INVALID_ARG;
    }

    // --- row pointers to the host: validation and SpMV plans
    std::vector<int32_t> rpa(m + 1), rpat(n + 1);
    MIP_HIP(hipMemcpyAsync(rpa.data(), lp.a_rowptr, (m + 1) * 4, hipMemcpyDeviceToHost, stream));
    MIP_HIP(hipMemcpyAsync(rpat.data(), lp.at_rowptr, (n + 1) * 4, hipMemcpyDeviceToHost, stream));
    MIP_HIP(hipStreamSynchronize(stream));
    int rc;
    if ((rc = check_rowptr(rpa, lp.m, nnz, "A"))) return rc;
    if ((rc = check_rowptr(rpat, lp.n, nnz, "A^T"))) return rc;
    S.hpa = make_plan(rpa, lp.m, o.lanes_a, o.long_row);
    S.hpat = make_plan(rpat, lp.n, o.lanes_at, o.long_row);
    if (!S.hpa.long_rows.empty())
        MIP_HIP(hipMemcpyAsync(w.long_a, S.hpa.long_rows.data(), S.hpa.long_rows.size() * 4,
                               hipMemcpyHostToDevice, stream));
    if (!S.hpat.long_rows.empty())
        MIP_HIP(hipMemcpyAsync(w.long_at, S.hpat.long_rows.data(), S.hpat.long_rows.size() * 4,
                               hipMemcpyHostToDevice, stream));
    S.pa = device_plan(S.hpa, lp.a_rowptr, w.long_a, lp.m);
    S.pat = device_plan(S.hpat, lp.at_rowptr, w.long_at, lp.n);
    {
        const int32_t tnz = tile_nnz_of(o), trows = tile_rows_of(o), srow = short_row_of(o);
        const int32_t tnz_t = tile_nnz_at_of(o), trows_t = tile_rows_at_of(o), srow_t = short_row_at_of(o);
        const std::vector<int32_t> ta = make_tile_desc(rpa, lp.m, tnz, trows),
                                   tat = make_tile_desc(rpat, lp.n, tnz_t, trows_t);
        if (!tile_desc_ok(ta, rpa, lp.m, tnz, trows) || !tile_desc_ok(tat, rpat, lp.n, tnz_t, trows_t))
            return set_error("internal: tile plan does not cover the rows"), MIPDHG_ERR_UNSUPPORTED;
        MIP_HIP(hipMemcpyAsync(w.tiles_a, ta.data(), ta.size() * 4, hipMemcpyHostToDevice, stream));
        MIP_HIP(hipMemcpyAsync(w.tiles_at, tat.data(), tat.size() * 4, hipMemcpyHostToDevice, stream));
        S.ta = make_tile_plan(lp.a_rowptr, w.tiles_a, (int32_t)(ta.size() / 4), lp.m, tnz, trows, srow);
        S.tat = make_tile_plan(lp.at_rowptr, w.tiles_at, (int32_t)(tat.size() / 4), lp.n, tnz_t, trows_t, srow_t);
        if ((rc = S.allow_tile_lds())) return rc;
        if ((rc = S.plan_persistent())) return rc;
        MIP_HIP(hipStreamSynchronize(stream));  // host vectors go out of scope
    }
    const int gta = S.ta.ntiles, gtat = S.tat.ntiles;
    const int64_t G = w.gcap;

    // --- validation: indices, finiteness, transpose consistency
    if (o.validate && (rc = validate_device(lp, S.ta, S.tat, w.flags, w.psetup, w.red, stream))) return rc;

    // --- norms of the original b and c
    double bn2 = 0, cn2 = 0;
    {
        const int gm = grid_for(m, 1024), gn = grid_for(n, 1024);
        hipLaunchKernelGGL(k_sumsq, dim3(gm), dim3(kBlock), 0, stream, lp.b, m, w.psetup);
        hipLaunchKernelGGL(k_reduce_rows, dim3(1), dim3(kBlock), 0, stream, (const double*)w.psetup, gm, 1, w.red);
        hipLaunchKernelGGL(k_sumsq, dim3(gn), dim3(kBlock), 0, stream, lp.c, n, w.psetup + G);
        hipLaunchKernelGGL(k_reduce_rows, dim3(1), dim3(kBlock), 0, stream,
                           (const double*)(w.psetup + G), gn, 1, w.red + 1);
        MIP_LAUNCH_CHECK();
    }

    // --- scaling: Ruiz passes, then one Pock-Chambolle pass
    hipLaunchKernelGGL(k_fill, dim3(grid_for(m)), dim3(kBlock), 0, stream, w.d_row, m, 1.0);
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kBlock), 0, stream, w.d_col, n, 1.0);
    MIP_LAUNCH_CHECK();
    const int passes = o.ruiz_iters + (o.pock_chambolle ? 1 : 0);
    for (int ps = 0; ps < passes; ++ps) {
        const bool maxmode = ps < o.ruiz_iters;
        if (maxmode) {
            hipLaunchKernelGGL((k_scale_stat<true>), dim3(gta), dim3(kBlock), tile_lds_bytes(S.ta, 8), stream, S.ta, lp.a_col, lp.a_val,
                               (const double*)w.d_row, (const double*)w.d_col, w.stat_r);
            hipLaunchKernelGGL((k_scale_stat<true>), dim3(gtat), dim3(kBlock), tile_lds_bytes(S.tat, 8), stream, S.tat, lp.at_col,
                               lp.at_val, (const double*)w.d_col, (const double*)w.d_row, w.stat_c);
        } else {
            hipLaunchKernelGGL((k_scale_stat<false>), dim3(gta), dim3(kBlock), tile_lds_bytes(S.ta, 8), stream, S.ta, lp.a_col, lp.a_val,
                               (const double*)w.d_row, (const double*)w.d_col, w.stat_r);
            hipLaunchKernelGGL((k_scale_stat<false>), dim3(gtat), dim3(kBlock), tile_lds_bytes(S.tat, 8), stream, S.tat, lp.at_col,
                               lp.at_val, (const double*)w.d_col, (const double*)w.d_row, w.stat_c);
        }
        hipLaunchKernelGGL(k_scale_update, dim3(grid_for(m)), dim3(kBlock), 0, stream, w.d_row,
                           (const double*)w.stat_r, m);
        hipLaunchKernelGGL(k_scale_update, dim3(grid_for(n)), dim3(kBlock), 0, stream, w.d_col,
                           (const double*)w.stat_c, n);
        MIP_LAUNCH_CHECK();
    }
    // scaled values in the iteration precision (sorted or row-major tile
    // layout), b~ and c~
    if (S.sorted()) {
        hipLaunchKernelGGL((k_sort_scale_tiles<V>), dim3(gta), dim3(kBlock), sort_lds_bytes(S.ta), stream, S.ta,
                           lp.a_col, lp.a_val, (const double*)w.d_row, (const double*)w.d_col, w.col_a, w.slot_a,
                           (V*)w.a_vs);
        hipLaunchKernelGGL((k_sort_scale_tiles<V>), dim3(gtat), dim3(kBlock), sort_lds_bytes(S.tat), stream, S.tat,
                           lp.at_col, lp.at_val, (const double*)w.d_col, (const double*)w.d_row, w.col_at, w.slot_at,
                           (V*)w.at_vs);
    } else {
        hipLaunchKernelGGL((k_scale_values<V>), dim3(grid_for(m * kWave, 4096)), dim3(kBlock), 0, stream,
                           lp.a_rowptr, lp.a_col, lp.a_val, (const double*)w.d_row, (const double*)w.d_col, lp.m,
                           (V*)w.a_vs);
        hipLaunchKernelGGL((k_scale_values<V>), dim3(grid_for(n * kWave, 4096)), dim3(kBlock), 0, stream,
                           lp.at_rowptr, lp.at_col, lp.at_val, (const double*)w.d_col, (const double*)w.d_row, lp.n,
                           (V*)w.at_vs);
    }
    // A's panel layout for the dual step (same scaled values as the copies) is
    // built on a second stream, so that its host-side steps overlap the power
    // iteration; the first stream waits for it before the loop
    struct SideStream {
        hipStream_t s = nullptr;
        hipEvent_t scaled = nullptr, built = nullptr;
        ~SideStream() {
            if (scaled) (void)hipEventDestroy(scaled);
            if (built) (void)hipEventDestroy(built);
            if (s) (void)hipStreamDestroy(s);
        }
    } side;
    if (S.panel()) {
        MIP_HIP(hipStreamCreateWithFlags(&side.s, hipStreamNonBlocking));
        MIP_HIP(hipEventCreateWithFlags(&side.scaled, hipEventDisableTiming));
        MIP_HIP(hipEventCreateWithFlags(&side.built, hipEventDisableTiming));
        MIP_HIP(hipEventRecord(side.scaled, stream));
        MIP_HIP(hipStreamWaitEvent(side.s, side.scaled, 0));
    }
    {
        const int gm = grid_for(m, 1024), gn = grid_for(n, 1024);
        hipLaunchKernelGGL((k_scale_vec<T>), dim3(gm), dim3(kBlock), 0, stream, lp.b, (const double*)w.d_row, m,
                           (T*)nullptr, w.psetup);
        hipLaunchKernelGGL(k_reduce_rows, dim3(1), dim3(kBlock), 0, stream, (const double*)w.psetup, gm, 1,
                           w.red + 2);
        hipLaunchKernelGGL((k_scale_vec<T>), dim3(gn), dim3(kBlock), 0, stream, lp.c, (const double*)w.d_col, n,
                           (T*)nullptr, w.psetup + G);
        hipLaunchKernelGGL(k_reduce_rows, dim3(1), dim3(kBlock), 0, stream,
                           (const double*)(w.psetup + G), gn, 1, w.red + 3);
        MIP_LAUNCH_CHECK();
    }

    if (has_bounds(lp)) {
        hipLaunchKernelGGL((k_scale_bounds<T>), dim3(grid_for(n)), dim3(kBlock), 0, stream, lp.lo, lp.hi,
                           (const double*)w.d_col, n, (T*)w.lo_t, (T*)w.hi_t);
        MIP_LAUNCH_CHECK();
    }

    // --- power iteration for sigma_hat = ||D_r A D_c||_2 (not for the
    // adaptive step, which starts from the largest scaled entry instead)
    if (!S.adaptive()) {
        const double v0 = 1.0 / sqrt((double)n);
        hipLaunchKernelGGL((k_fill_t<T>), dim3(grid_for(n)), dim3(kBlock), 0, stream, (T*)w.pv, n, (T)v0);
        // on the scaled iteration copies (tile plans with their layout)
        TilePlan pa = S.ta, pat = S.tat;
        const bool srt = S.sorted();
        if (srt) {
            pa.slot = w.slot_a;
            pat.slot = w.slot_at;
        }
        const int32_t* ca = srt ? w.col_a : lp.a_col;
        const int32_t* cat = srt ? w.col_at : lp.at_col;
        // vectors in the iterate type T (the buffers hold float64 room)
        auto spmv = [&](const TilePlan& tp, const int32_t* col, const void* vals, const void* xv, void* yv,
                        double* part) {
            const T* x = (const T*)xv;
            T* y = (T*)yv;
            const bool big = tp.tile_nnz > 8 * kBlock;
            const dim3 g(tp.ntiles), b(kBlock);
            const size_t lds = tile_lds_bytes(tp, 8);
            if (srt && big) hipLaunchKernelGGL((k_spmv_copy<V, true, T, 16>), g, b, lds, stream, tp, col, (const V*)vals, x, y, part);
            else if (srt) hipLaunchKernelGGL((k_spmv_copy<V, true, T, 8>), g, b, lds, stream, tp, col, (const V*)vals, x, y, part);
            else if (big) hipLaunchKernelGGL((k_spmv_copy<V, false, T, 16>), g, b, lds, stream, tp, col, (const V*)vals, x, y, part);
            else hipLaunchKernelGGL((k_spmv_copy<V, false, T, 8>), g, b, lds, stream, tp, col, (const V*)vals, x, y, part);
        };
        for (int k = 0; k <= o.power_iters; ++k) {
            // av = A~ v, hist[k] = ||av||^2
            spmv(pa, ca, w.a_vs, w.pv, w.pav, w.psetup);
            hipLaunchKernelGGL(k_reduce_rows, dim3(1), dim3(kBlock), 0, stream, (const double*)w.psetup, gta, 1,
                               w.hist + k);
            if (k == o.power_iters) break;
            // u = A~^T av, v = u / ||u||
            spmv(pat, cat, w.at_vs, w.pav, w.pu, w.psetup + G);
            hipLaunchKernelGGL((k_normalize<T>), dim3(grid_for(n, 1024)), dim3(kBlock), 0, stream, (const T*)w.pu,
                               (T*)w.pv, n, (const double*)(w.psetup + G), gtat);
            MIP_LAUNCH_CHECK();
        }
        MIP_LAUNCH_CHECK();
    }
    if (S.panel()) {
        rc = panel_build<V>(rpa, lp.m, lp.n, nnz, lp.a_rowptr, lp.a_col, lp.a_val, (const double*)w.d_row,
                            (const double*)w.d_col, S.panel_w(), sizeof(T), w.pl, side.s);
        if (rc) {
            (void)hipStreamSynchronize(side.s);
            (void)hipStreamSynchronize(stream);
            return rc;
        }
        if (S.rowpanel()) {
            int dev = 0, cus = 256;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
                cus = 256;
            rc = rowpanel_build<V>(rpat, lp.n, lp.m, nnz, lp.at_rowptr, lp.at_col, lp.at_val, lp.a_rowptr, lp.a_col,
                                   (const double*)w.d_col, (const double*)w.d_row, S.panel_w(), cus, w.rl, side.s);
            if (rc) {
                (void)hipStreamSynchronize(side.s);
                (void)hipStreamSynchronize(stream);
                return rc;
            }
        }
        MIP_HIP(hipEventRecord(side.built, side.s));
        MIP_HIP(hipStreamWaitEvent(stream, side.built, 0));
    }
    if (S.adaptive()) {  // max_ij |A~_ij| from the row maxima of the scaled matrix
        hipLaunchKernelGGL((k_scale_stat<true>), dim3(gta), dim3(kBlock), tile_lds_bytes(S.ta, 8), stream, S.ta,
                           lp.a_col, lp.a_val, (const double*)w.d_row, (const double*)w.d_col, w.stat_r);
        const int gmx = grid_for(m);
        hipLaunchKernelGGL(k_max_part, dim3(gmx), dim3(kBlock), 0, stream, (const double*)w.stat_r, m, w.psetup);
        hipLaunchKernelGGL(k_max_part, dim3(1), dim3(kBlock), 0, stream, (const double*)w.psetup, (int64_t)gmx,
                           w.red + 4);
        MIP_LAUNCH_CHECK();
    }
    std::vector<double> hist(S.adaptive() ? 1 : o.power_iters + 1, 0.0);
    double red[5];
    if (!S.adaptive()) MIP_HIP(hipMemcpyAsync(hist.data(), w.hist, hist.size() * 8, hipMemcpyDeviceToHost, stream));
    MIP_HIP(hipMemcpyAsync(red, w.red, 5 * 8, hipMemcpyDeviceToHost, stream));
    MIP_HIP(hipStreamSynchronize(stream));
    bn2 = red[0];
    cn2 = red[1];
    for (auto& h : hist) h = sqrt(h);
    const double sigma_hat = hist.back();
    double eta;
    if (S.adaptive()) {
        eta = o.step0 > 0.0 ? o.step0 : (red[4] > 0.0 ? 1.0 / red[4] : 1.0);
    } else if (sigma_hat <= 0.0) {
        eta = o.step_safety;
    } else if (o.pock_chambolle && hist.size() > 10 &&
               fabs(hist.back() - hist[hist.size() - 11]) > 1e-3 * hist.back()) {
        eta = o.step_safety;
    } else {
        eta = o.step_safety / sigma_hat;
    }
    const double nbt = sqrt(red[2]), nct = sqrt(red[3]);
    const double omega0 = (nbt > 1e-10 && nct > 1e-10) ? nct / nbt : 1.0;

    // --- control block and initial point (or, when resuming, the
    // workspace's own state, checked against this problem and layout)
    if (o.resume) {
        Ctrl cur;
        MIP_HIP(hipMemcpyAsync(&cur, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
        MIP_HIP(hipStreamSynchronize(stream));
        // the data, by the norms of b and c and the step size that setup has
        // just recomputed (setup leaves the iterates and the control block)
        if (cur.b_norm != sqrt(bn2) || cur.c_norm != sqrt(cn2) || cur.eta0 != eta)
            return set_error("resume: the workspace holds the state of another LP of these sizes"),
                   MIPDHG_ERR_INVALID_ARG;
        // a solve that stopped at an evaluation (optimal or at its iteration
        // limit) skipped that evaluation's restart decision: take it again
        // with the new tolerance and limit
        const bool redo = cur.status != ST_RUNNING;
        if (redo) cur.t_base -= cur.last_nit;
        cur.status = ST_RUNNING;
        cur.eps = eps;
        cur.max_iter = o.max_iter;
        cur.infeas_tol = o.infeas_tol;
        MIP_HIP(hipMemcpyAsync(w.ctrl, &cur, sizeof(Ctrl), hipMemcpyHostToDevice, stream));
        if (redo && (rc = S.launch_decide(cur.last_nit))) return rc;
        MIP_HIP(hipStreamSynchronize(stream));
    }
    Ctrl c0;
    memset(&c0, 0, sizeof(c0));
    c0.omega = omega0;
    c0.eta = eta;
    c0.tau = eta / omega0;
    c0.sigma = eta * omega0;
    c0.k_base = 0;
    c0.t_base = 0;
    c0.status = ST_RUNNING;
    c0.restart_now = 0;
    c0.R0 = NAN;
    c0.R_prev = INFINITY;
    c0.eps = eps;
    c0.b_norm = sqrt(bn2);
    c0.c_norm = sqrt(cn2);
    c0.beta_suff = o.beta_suff;
    c0.beta_nec = o.beta_nec;
    c0.beta_art = o.beta_art;
    c0.pw_theta = o.pw_theta;
    c0.pw_ki = o.pw_ki;
    c0.pw_kd = o.pw_kd;
    c0.pw_int = 0.0;
    c0.pw_err = 0.0;
    c0.pw_count = 0;
    c0.max_iter = o.max_iter;
    c0.do_restarts = o.restarts;
    c0.resumable = 1;
    c0.fingerprint = fp;
    c0.have_prev = 0;
    c0.infeas_tol = o.infeas_tol;
    c0.eta0 = eta;
    c0.step_rule = o.step_rule;
    c0.accepted = 1;
    c0.rejected = 0;
    if (!o.resume) {
        MIP_HIP(hipMemcpyAsync(w.ctrl, &c0, sizeof(Ctrl), hipMemcpyHostToDevice, stream));
        hipLaunchKernelGGL((k_init_state<T>), dim3(grid_for(n)), dim3(kBlock), 0, stream, o.x_init,
                           (const double*)w.d_col, n, (T*)w.x, (T*)w.x0, (T*)w.xhat);
        hipLaunchKernelGGL((k_init_state<T>), dim3(grid_for(m)), dim3(kBlock), 0, stream, o.y_init,
                           (const double*)w.d_row, m, (T*)w.y, (T*)w.y0, (T*)w.yhat);
        MIP_LAUNCH_CHECK();
        if ((rc = S.launch_anchor_resid(1))) return rc;
        hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kBlock), 0, stream, w.xprev, n, 0.0);
        hipLaunchKernelGGL(k_fill, dim3(grid_for(m)), dim3(kBlock), 0, stream, w.yprev, m, 0.0);
        if (S.adaptive())  // x = x0: A~ (x - x0) = 0
            hipLaunchKernelGGL((k_fill_t<T>), dim3(grid_for(m)), dim3(kBlock), 0, stream, (T*)w.ax, m, (T)0);
        hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kBlock), 0, stream, w.atyprev, n, 0.0);
        hipLaunchKernelGGL(k_fill, dim3(grid_for(m)), dim3(kBlock), 0, stream, w.axprev, m, 0.0);
        MIP_LAUNCH_CHECK();
    }
    MIP_HIP(hipStreamSynchronize(stream));
    const auto t1 = clk::now();

    // --- main loop
    const int E = o.eval_every;
    const bool trace = o.trace_iters > 0;
    const bool graph = o.use_graph && !trace && o.kernel_timing != 1;
    if (o.kernel_timing == 1) {
        S.timing = true;
        S.tev.resize(3 * (size_t)E);
        for (auto& e : S.tev) MIP_HIP(hipEventCreate(&e));
    }
    // host objects of the loop, released on every return path (after the
    // stream has been synchronised on the normal one)
    // blocks in flight: one running and one queued behind it, so that the GPU
    // never waits for the host, and one block (returning at once) runs past
    // the one that ends the solve
    constexpr int kDepth = 2;
    struct LoopRes {
        hipGraphExec_t gexec = nullptr;
        hipGraph_t g = nullptr;
        hipStream_t cap = nullptr;
        Ctrl* ring = nullptr;  // pinned ring of status words, one per block in flight
        hipEvent_t ev[kDepth] = {};
        ~LoopRes() {
            for (auto e : ev)
                if (e) (void)hipEventDestroy(e);
            if (ring) (void)hipHostFree(ring);
            if (gexec) (void)hipGraphExecDestroy(gexec);
            if (g) (void)hipGraphDestroy(g);
            if (cap) (void)hipStreamDestroy(cap);
        }
    } res;
    double ms_graph = 0.0;
    if (graph && o.max_iter >= E) {
        const auto tg = clk::now();
        MIP_HIP(hipStreamCreateWithFlags(&res.cap, hipStreamNonBlocking));
        S.stream = res.cap;
        MIP_HIP(hipStreamBeginCapture(res.cap, hipStreamCaptureModeThreadLocal));
        rc = S.enqueue_block(E, 1, false);
        hipError_t ce = hipStreamEndCapture(res.cap, &res.g);
        S.stream = stream;
        if (rc) return rc;
        MIP_HIP(ce);
        MIP_HIP(hipGraphInstantiate(&res.gexec, res.g, nullptr, nullptr, 0));
        ms_graph = std::chrono::duration<double, std::milli>(clk::now() - tg).count();
    }
    MIP_HIP(hipHostMalloc((void**)&res.ring, sizeof(Ctrl) * kDepth, hipHostMallocDefault));
    for (int i = 0; i < kDepth; ++i) MIP_HIP(hipEventCreateWithFlags(&res.ev[i], hipEventDisableTiming));
    Ctrl* const ring = res.ring;
    hipEvent_t* const ev = res.ev;
    const hipGraphExec_t gexec = res.gexec;
    int64_t launched = 0;
    if (o.resume) {
        Ctrl cur;
        MIP_HIP(hipMemcpyAsync(&cur, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
        MIP_HIP(hipStreamSynchronize(stream));
        launched = cur.t_base;  // iterations already done
        if (cur.status != ST_RUNNING) launched = o.max_iter;  // decided at once (e.g. still optimal)
    }
    int64_t blocks = 0, checked = 0;
    bool done = false, timed_out = false;
    rc = 0;
    while (!done && launched < o.max_iter) {
        const int nit = (int)std::min<int64_t>(E, o.max_iter - launched);
        if (gexec && nit == E) {
            if (hipGraphLaunch(gexec, stream) != hipSuccess) {
                set_error("hipGraphLaunch failed");
                rc = MIPDHG_ERR_HIP;
                break;
            }
        } else if ((rc = S.enqueue_block(nit, launched + 1, trace))) {
            break;
        }
        launched += nit;
        const int slot = (int)(blocks % kDepth);
        if (hipMemcpyAsync(ring + slot, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipEventRecord(ev[slot], stream) != hipSuccess) {
            set_error("status copy failed");
            rc = MIPDHG_ERR_HIP;
            break;
        }
        ++blocks;
        // keep kDepth-1 blocks queued; look at the oldest one
        while (checked < blocks && (blocks - checked >= kDepth || trace || S.timing || launched >= o.max_iter)) {
            const int cs = (int)(checked % kDepth);
            if (hipEventSynchronize(ev[cs]) != hipSuccess) {
                set_error("hipEventSynchronize failed");
                rc = MIPDHG_ERR_HIP;
                done = true;
                break;
            }
            ++checked;
            if (ring[cs].status != ST_RUNNING) {
                done = true;
                break;
            }
        }
        if (!done && o.time_limit_s < 1e300 &&
            std::chrono::duration<double>(clk::now() - t0).count() > o.time_limit_s) {
            timed_out = true;
            break;
        }
    }
    hipError_t se = hipStreamSynchronize(stream);
    const auto t2 = clk::now();
    if (rc) return rc;
    MIP_HIP(se);

    Ctrl cf;
    MIP_HIP(hipMemcpy(&cf, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    if (o.kernel_timing == 2) {
        // back-to-back runs of each iteration kernel between two events; the
        // control word is set to running for the runs (a finished solve makes
        // the kernels skip their row sums) and restored afterwards
        constexpr int R = 256;
        S.tev.assign(3, nullptr);  // the solver releases its events
        for (auto& e : S.tev) MIP_HIP(hipEventCreate(&e));
        hipEvent_t* const te = S.tev.data();
        const int32_t running = ST_RUNNING;
        MIP_HIP(hipMemcpyAsync(&w.ctrl->status, &running, sizeof(int32_t), hipMemcpyHostToDevice, stream));
        S.stream = stream;
        MIP_HIP(hipEventRecord(te[0], stream));
        for (int r = 0; r < R && !rc; ++r) rc = S.launch_primal(1, 0);
        MIP_HIP(hipEventRecord(te[1], stream));
        for (int r = 0; r < R && !rc; ++r) rc = S.launch_dual(1, 0);
        MIP_HIP(hipEventRecord(te[2], stream));
        MIP_HIP(hipMemcpyAsync(&w.ctrl->status, &cf.status, sizeof(int32_t), hipMemcpyHostToDevice, stream));
        const int32_t no = 0;  // the timing runs moved the iterates: not resumable
        MIP_HIP(hipMemcpyAsync(&w.ctrl->resumable, &no, sizeof(int32_t), hipMemcpyHostToDevice, stream));
        MIP_HIP(hipStreamSynchronize(stream));
        float a = 0.f, b = 0.f;
        MIP_HIP(hipEventElapsedTime(&a, te[0], te[1]));
        MIP_HIP(hipEventElapsedTime(&b, te[1], te[2]));
        if (rc) return rc;
        S.ms_p = a;
        S.ms_d = b;
        S.n_p = S.n_d = R;
    }
    int status = cf.status;
    if (status == ST_RUNNING) status = timed_out ? MIPDHG_TIME_LIMIT : MIPDHG_ITER_LIMIT;
    if (d_row) MIP_HIP(hipMemcpyAsync(d_row, w.d_row, m * 8, hipMemcpyDeviceToDevice, stream));
    if (d_col) MIP_HIP(hipMemcpyAsync(d_col, w.d_col, n * 8, hipMemcpyDeviceToDevice, stream));
    MIP_HIP(hipStreamSynchronize(stream));
    const auto t3 = clk::now();
    if (info) {
        memset(info, 0, sizeof(*info));
        info->status = status;
        info->restarts = cf.restarts;
        info->iters = cf.eval_t;
        info->rp_norm = sqrt(cf.rp2);
        info->rd_norm = sqrt(cf.rd2);
        info->pobj = cf.pobj;
        info->dobj = cf.dobj;
        info->gap = fabs(cf.pobj - cf.dobj);
        info->b_norm = c0.b_norm;
        info->c_norm = c0.c_norm;
        info->rel_rp = info->rp_norm / (1.0 + c0.b_norm);
        info->rel_rd = info->rd_norm / (1.0 + c0.c_norm);
        info->rel_gap = info->gap / (1.0 + fabs(cf.pobj) + fabs(cf.dobj));
        info->rp_inf = cf.rp_inf;
        info->rd_inf = cf.rd_inf;
        info->xz = cf.xz;
        info->max_violation = std::max(std::max(cf.rp_inf, cf.rd_inf), cf.xz / (1.0 + fabs(cf.pobj)));
        info->sigma_hat = sigma_hat;
        info->eta = o.step_rule == 1 ? cf.eta : eta;
        info->rejected = cf.rejected;
        info->omega0 = omega0;
        info->omega = cf.omega;
        info->ms_setup = std::chrono::duration<double, std::milli>(t1 - t0).count();
        info->ms_iter = std::chrono::duration<double, std::milli>(t2 - t1).count();
        info->ms_total = std::chrono::duration<double, std::milli>(t3 - t0).count();
        const double vs = sizeof(V), ts = sizeof(T);
        // per iteration: A and A^T values + indices, row pointers, gathers,
        // streamed vectors (primal: u, x0, r_c read, u, x_bar - x0 written;
        // dual: v, r_b read, v written)
        // general form: the primal reads two scaled bounds per column, the
        // dual its anchor and one sense byte per row
        info->bytes_primal = nnz * (vs + 4.0) + 4.0 * (n + 1) + ts * (double)m + (has_bounds(lp) ? 7.0 : 5.0) * ts * n;
        info->bytes_dual = nnz * (vs + 4.0) + 4.0 * (m + 1) + ts * (double)n + 3.0 * ts * m +
                           (has_sense(lp) ? (ts + 1.0) * m : 0.0);
        info->bytes_per_iter = info->bytes_primal + info->bytes_dual;
        info->ms_primal = S.n_p ? S.ms_p / S.n_p : 0.0;
        info->ms_dual = S.n_d ? S.ms_d / S.n_d : 0.0;
        info->n_primal = S.n_p;
        info->n_dual = S.n_d;
        info->lanes_a = S.hpa.lanes;
        info->lanes_at = S.hpat.lanes;
        info->long_a = (int32_t)S.hpa.long_rows.size();
        info->long_at = (int32_t)S.hpat.long_rows.size();
        info->ms_graph = ms_graph;
    }
    return status;
}

}  // namespace mip

namespace mip {

// The parts of the workspace a resumed solve continues from, as (offset,
// bytes) pairs in the workspace layout of these LP sizes and options.
static std::vector<std::pair<size_t, size_t>> state_regions(const mipdhg_lp& lp, const mipdhg_options& o) {
    char* const base = reinterpret_cast<char*>(uintptr_t(4096));  // layout only, never dereferenced
    const PlainWs w = carve(base, 0, lp.m, lp.n, lp.nnz, o.precision, o.power_iters, tile_nnz_of(o), tile_rows_of(o),
                            tile_nnz_at_of(o), tile_rows_at_of(o), sorted_layout(o, lp.m, lp.n), has_bounds(lp),
                            o.restart_avg != 0, o.spmv_kind >= 3, o.step_rule == 1, o.spmv_kind == 4);
    const size_t ts = (o.precision == MIPDHG_FP64 || o.precision == MIPDHG_FP32_A) ? 8 : 4;
    const size_t m = (size_t)lp.m, n = (size_t)lp.n, G = (size_t)w.gcap;
    auto at = [&](const void* p, size_t bytes) { return std::make_pair((size_t)((const char*)p - base), bytes); };
    std::vector<std::pair<size_t, size_t>> r = {
        at(w.ctrl, sizeof(Ctrl)),      at(w.pp, G * 3 * 8),          at(w.pd, G * 3 * 8),
        at(w.per, G * kEvalRowsW * 8), at(w.pec, G * kEvalColsW * 8), at(w.xprev, n * 8),
        at(w.yprev, m * 8),            at(w.axprev, m * 8),          at(w.atyprev, n * 8),
        at(w.x, n * ts),               at(w.x0, n * ts),             at(w.xhat, n * ts),
        at(w.y, m * ts),               at(w.y0, m * ts),             at(w.yhat, m * ts),
        at(w.ct, n * ts),              at(w.bt, m * ts)};
    if (o.restart_avg) {
        r.push_back(at(w.x_avg, n * ts));
        r.push_back(at(w.y_avg, m * ts));
    }
    if (o.step_rule == 1) r.push_back(at(w.ax, m * ts));  // between blocks the iterate is in the first buffers
    return r;
}

static int state_copy(const mipdhg_lp* lp, const mipdhg_options* opt, char* ws, size_t ws_bytes, char* buf,
                      size_t buf_bytes, bool out, hipStream_t stream) {
    clear_error();
    int rc = check_lp(lp);
    if (rc) return rc;
    if (!opt || !ws || !buf) return set_error("NULL argument"), MIPDHG_ERR_INVALID_ARG;
    if ((rc = check_options(opt))) return rc;
    size_t need = 0;
    if ((rc = mipdhg_workspace_size(lp, opt, &need))) return rc;
    if (ws_bytes < need) return set_error("workspace too small: %zu bytes, %zu needed", ws_bytes, need), MIPDHG_ERR_WORKSPACE;
    const auto regions = state_regions(*lp, *opt);
    size_t total = 0;
    for (const auto& r : regions) total += r.second;
    if (buf_bytes < total)
        return set_error("state buffer too small: %zu bytes, %zu needed", buf_bytes, total), MIPDHG_ERR_INVALID_ARG;
    size_t pos = 0;
    for (const auto& r : regions) {
        if (out) MIP_HIP(hipMemcpyAsync(buf + pos, ws + r.first, r.second, hipMemcpyDefault, stream));
        else MIP_HIP(hipMemcpyAsync(ws + r.first, buf + pos, r.second, hipMemcpyDefault, stream));
        pos += r.second;
    }
    MIP_HIP(hipStreamSynchronize(stream));
    return 0;
}

}  // namespace mip

extern "C" int mipdhg_state_size(const mipdhg_lp* lp, const mipdhg_options* opt, size_t* bytes) {
    clear_error();
    int rc = check_lp(lp);
    if (rc) return rc;
    if (!opt || !bytes) return set_error("NULL argument"), MIPDHG_ERR_INVALID_ARG;
    if ((rc = check_options(opt))) return rc;
    size_t total = 0;
    for (const auto& r : state_regions(*lp, *opt)) total += r.second;
    *bytes = total;
    return 0;
}

extern "C" int mipdhg_state_export(const mipdhg_lp* lp, const mipdhg_options* opt, const void* workspace,
                                   size_t workspace_bytes, void* dst, size_t dst_bytes, void* stream) {
    return state_copy(lp, opt, (char*)workspace, workspace_bytes, (char*)dst, dst_bytes, true, (hipStream_t)stream);
}

extern "C" int mipdhg_state_import(const mipdhg_lp* lp, const mipdhg_options* opt, void* workspace,
                                   size_t workspace_bytes, const void* src, size_t src_bytes, void* stream) {
    return state_copy(lp, opt, (char*)workspace, workspace_bytes, (char*)src, src_bytes, false, (hipStream_t)stream);
}

extern "C" int mipdhg_solve(const mipdhg_lp* lp, const mipdhg_options* opt, double eps_rel, void* workspace,
                            size_t workspace_bytes, void* stream, double* x, double* y, double* z, double* r_p,
                            double* r_d, double* d_row, double* d_col, mipdhg_info* info) {
    clear_error();
    int rc = check_lp(lp);
    if (rc) return rc;
    if (!opt) return set_error("options are NULL"), MIPDHG_ERR_INVALID_ARG;
    if ((rc = check_options(opt))) return rc;
    if (!(eps_rel >= 0.0) || !std::isfinite(eps_rel)) return set_error("eps_rel must be finite and >= 0"), MIPDHG_ERR_INVALID_ARG;
    if (!workspace || !x || !y || !z || !r_p || !r_d) return set_error("workspace and all five outputs are required"), MIPDHG_ERR_INVALID_ARG;
    if (is_general(*lp) && opt->spmv_kind == 1)
        return set_error("the general form runs on the tile kernels (spmv_kind 0 or 2)"), MIPDHG_ERR_UNSUPPORTED;
    if (opt->restart_avg && opt->spmv_kind != 0)
        return set_error("restart to average runs on the one-workgroup-per-tile kernels (spmv_kind 0)"),
               MIPDHG_ERR_UNSUPPORTED;
    if (opt->step_rule == 1 && opt->spmv_kind != 0)
        return set_error("the adaptive step runs on the one-workgroup-per-tile kernels (spmv_kind 0)"),
               MIPDHG_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    switch (opt->precision) {
        case MIPDHG_FP64:
            return solve_impl<double, double, double>(*lp, *opt, eps_rel, workspace, workspace_bytes, s, x, y, z, r_p,
                                                      r_d, d_row, d_col, info);
        case MIPDHG_FP32:
            return solve_impl<float, float, double>(*lp, *opt, eps_rel, workspace, workspace_bytes, s, x, y, z, r_p,
                                                    r_d, d_row, d_col, info);
        case MIPDHG_FP32_BF16A:
            return solve_impl<float, uint16_t, double>(*lp, *opt, eps_rel, workspace, workspace_bytes, s, x, y, z,
                                                       r_p, r_d, d_row, d_col, info);
        case MIPDHG_FP32_A:
            return solve_impl<double, float, double>(*lp, *opt, eps_rel, workspace, workspace_bytes, s, x, y, z, r_p,
                                                     r_d, d_row, d_col, info);
        default:
            return solve_impl<float, float, float>(*lp, *opt, eps_rel, workspace, workspace_bytes, s, x, y, z, r_p,
                                                   r_d, d_row, d_col, info);
    }
}
