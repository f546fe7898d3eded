// Builder of the panel layout (panel.h): row groups and panels on the host
// from each row's column span, the per-(row, panel) counts, the chunks and
// the scaled values on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "common.h"
#include "panel.h"
#include "plain.h"

namespace mip {

namespace {

// smallest and largest column of every row (an empty row: lo > hi)
__global__ void k_row_span(const int32_t* rowptr, const int32_t* col, int32_t nrows, int32_t* span) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * blockDim.x) {
        int32_t lo = 0x7fffffff, hi = -1;
        for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) {
            const int32_t c = col[k];
            lo = c < lo ? c : lo;
            hi = c > hi ? c : hi;
        }
        span[2 * r] = lo;
        span[2 * r + 1] = hi;
    }
}

__device__ __forceinline__ int64_t seg_of(const PanelGroup& g, int p, int32_t r) {
    return g.seg_base + (int64_t)p * (g.r1 - g.r0) + (r - g.r0);
}

// nonzeros of every row in every panel of its group (one thread per row)
__global__ void k_seg_count(const int32_t* rowptr, const int32_t* col, int32_t nrows, const int32_t* row_group,
                            const PanelGroup* groups, int width, int32_t* counts) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * blockDim.x) {
        const PanelGroup g = groups[row_group[r]];
        for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) ++counts[seg_of(g, (col[k] - g.lo) / width, (int32_t)r)];
    }
}

// One thread per unit walks the group's rows and cuts the unit's row parts
// into chunks of at most kPanelChunk nonzeros that end at a row end.  FILL
// false: the unit's number of chunks and padded elements; FILL true: the
// chunk descriptors, every part's first element and row inside its chunk,
// and the padding (value 0, column 0).
template <bool FILL, typename V>
__global__ void k_unit_chunks(const PanelGroup* groups, const int32_t* unit_group, const int32_t* unit_panel,
                              int32_t nunits, const int32_t* counts, int32_t* nch, int64_t* nel,
                              const int32_t* ch_off, const int64_t* el_off, PanelChunk* chunks, int32_t* seg_off,
                              uint16_t* seg_rid, V* val, uint16_t* colv, uint16_t* rid, int32_t* err) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nunits) return;
    const PanelGroup g = groups[unit_group[u]];
    const int p = unit_panel[u];
    int32_t c = FILL ? ch_off[u] : 0;
    int64_t e = FILL ? el_off[u] : 0;
    int cnt = 0, row0 = -1;
    auto close = [&]() {
        if (cnt == 0) return;
        if (FILL) {
            chunks[c] = PanelChunk{(int32_t)e, cnt, row0, u};
            for (int q = cnt; q < ((cnt + 7) & ~7); ++q) {
                val[e + q] = (V)0;
                colv[e + q] = 0;
                rid[e + q] = 0;
            }
        }
        ++c;
        e += (cnt + 7) & ~7;
        cnt = 0;
        row0 = -1;
    };
    // the unit's counts are contiguous over the rows: read 16 at a time (the
    // loads issued together) and walk them in order
    const int64_t sb = seg_of(g, p, g.r0);
    for (int32_t rb = g.r0; rb < g.r1; rb += 16) {
        int lens[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) lens[q] = rb + q < g.r1 ? counts[sb + (rb - g.r0) + q] : 0;
        for (int q = 0; q < 16; ++q) {
            const int len = lens[q];
            if (len == 0) continue;
            const int32_t r = rb + q;
            if (len > kPanelChunk) {
                atomicOr(err, 1);
                return;
            }
            if (cnt + len > kPanelChunk) close();
            if (row0 < 0) row0 = r;
            if (FILL) {
                const int64_t s = sb + (r - g.r0);
                seg_off[s] = (int32_t)(e + cnt);
                seg_rid[s] = (uint16_t)(r - row0);
            }
            cnt += len;
        }
    }
    close();
    if (!FILL) {
        nch[u] = c;
        nel[u] = e;
    }
}

// scaled values, columns inside the panel and row indices, one thread per row
// (cursor: the part's running count, zeroed beforehand)
template <typename V>
__global__ void k_panel_scatter(const int32_t* rowptr, const int32_t* col, const double* val, const double* d_self,
                                const double* d_other, int32_t nrows, const int32_t* row_group,
                                const PanelGroup* groups, int width, const int32_t* seg_off, const uint16_t* seg_rid,
                                int32_t* cursor, V* out, uint16_t* colv, uint16_t* rid) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * blockDim.x) {
        const PanelGroup g = groups[row_group[r]];
        const double ds = d_self[r];
        for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) {
            const int32_t cc = col[k];
            const int p = (cc - g.lo) / width;
            const int64_t s = seg_of(g, p, (int32_t)r);
            const int64_t pos = seg_off[s] + cursor[s]++;
            const double v = ds * val[k] * d_other[cc];  // the tile copies' expression
            if constexpr (sizeof(V) == 2) {
                out[pos] = f32_to_bf16_rne((float)v);
            } else {
                out[pos] = (V)v;
            }
            colv[pos] = (uint16_t)(cc - g.lo - p * width);
            rid[pos] = seg_rid[s];
        }
    }
}

}  // namespace

template <typename V>
int panel_build(const std::vector<int32_t>& rp, int32_t nrows, int32_t ncols, int64_t nnz, const int32_t* rowptr,
                const int32_t* col, const double* val, const double* d_self, const double* d_other, int width,
                size_t partial_elem_bytes, PanelLayout& L, hipStream_t stream) {
    (void)ncols;
    const int64_t seg_cap = panel_seg_cap(nrows, nnz);
    if (seg_cap < 2 * (int64_t)nrows) return set_error("internal: panel segment capacity"), MIPDHG_ERR_UNSUPPORTED;
    // --- every row's column span (through the counts array, not yet in use)
    hipLaunchKernelGGL(k_row_span, dim3(grid_for(nrows)), dim3(kBlock), 0, stream, rowptr, col, nrows, L.counts);
    MIP_LAUNCH_CHECK();
    std::vector<int32_t> span(2 * (size_t)nrows);
    MIP_HIP(hipMemcpyAsync(span.data(), L.counts, span.size() * 4, hipMemcpyDeviceToHost, stream));
    MIP_HIP(hipStreamSynchronize(stream));
    // --- groups of consecutive rows: "narrow" rows (span within 4 panels)
    // while the group's span stays within 4 panels; "wide" rows together;
    // empty rows join the group they fall in
    const int64_t span_max = 4 * (int64_t)width;
    constexpr int64_t kNarrowNnz = 1 << 20, kWideNnz = 1 << 22;
    std::vector<PanelGroup> groups;
    std::vector<int32_t> row_group(nrows);
    struct Open {
        int32_t r0 = 0, lo = 0, hi = -1;
        int64_t nnz = 0;
        int kind = -1;  // -1 empty so far, 0 narrow, 1 wide
    } cur;
    auto flush = [&](int32_t r_end) {
        if (r_end <= cur.r0) return;
        PanelGroup g;
        g.r0 = cur.r0;
        g.r1 = r_end;
        g.lo = cur.hi >= cur.lo ? cur.lo & ~7 : 0;  // a multiple of 8: aligned vector loads of a panel
        g.np = cur.hi >= cur.lo ? (int32_t)((cur.hi - g.lo) / width + 1) : 0;
        g.seg_base = 0;
        groups.push_back(g);
    };
    for (int32_t r = 0; r < nrows; ++r) {
        const int32_t lo = span[2 * r], hi = span[2 * r + 1];
        const int64_t len = rp[r + 1] - rp[r];
        const bool rows_full = r - cur.r0 >= kPanelMaxGroupRows;
        if (len == 0) {
            if (rows_full) {
                flush(r);
                cur = Open();
                cur.r0 = r;
            }
            row_group[r] = (int32_t)groups.size();
            continue;
        }
        const int kind = (int64_t)hi - (lo & ~7) + 1 > span_max ? 1 : 0;  // spans from the aligned start
        bool join = !rows_full && (cur.kind < 0 || cur.kind == kind);
        if (join && cur.kind >= 0) {
            const int64_t nlo = std::min(cur.lo, lo), nhi = std::max(cur.hi, hi);
            if (kind == 0) join = nhi - (nlo & ~7) + 1 <= span_max && cur.nnz + len <= kNarrowNnz;
            else join = cur.nnz + len <= kWideNnz;
        }
        if (!join) {
            flush(r);
            cur = Open();
            cur.r0 = r;
        }
        if (cur.kind < 0) {
            cur.kind = kind;
            cur.lo = lo;
            cur.hi = hi;
        } else {
            cur.lo = std::min(cur.lo, lo);
            cur.hi = std::max(cur.hi, hi);
        }
        cur.nnz += len;
        row_group[r] = (int32_t)groups.size();
    }
    flush(nrows);
    int64_t nseg = 0;
    std::vector<int32_t> unit_group, unit_panel;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        PanelGroup& g = groups[gi];
        g.seg_base = nseg;
        nseg += (int64_t)(g.r1 - g.r0) * g.np;
        for (int p = 0; p < g.np; ++p) {
            unit_group.push_back((int32_t)gi);
            unit_panel.push_back(p);
        }
    }
    if (nseg > seg_cap || (int64_t)unit_group.size() > kPanelMaxUnits || (int64_t)groups.size() > kPanelMaxUnits)
        return set_error("panel layout: %lld row parts or %zu units exceed the workspace's capacity",
                         (long long)nseg, unit_group.size()),
               MIPDHG_ERR_UNSUPPORTED;
    const int32_t nunits = (int32_t)unit_group.size();
    L.ngroups = (int32_t)groups.size();
    L.nseg = nseg;
    // --- device tables; per-part counts
    MIP_HIP(hipMemcpyAsync(L.groups, groups.data(), groups.size() * sizeof(PanelGroup), hipMemcpyHostToDevice, stream));
    MIP_HIP(hipMemcpyAsync(L.row_group, row_group.data(), (size_t)nrows * 4, hipMemcpyHostToDevice, stream));
    std::vector<int32_t> wide;
    for (const PanelGroup& g : groups)
        if (g.np > kPanelWideRow)
            for (int32_t r = g.r0; r < g.r1; ++r) wide.push_back(r);
    L.nwide = (int32_t)wide.size();
    if (!wide.empty())
        MIP_HIP(hipMemcpyAsync(L.wide_rows, wide.data(), wide.size() * 4, hipMemcpyHostToDevice, stream));
    // unit tables for the build live in the chunk array's space (rebuilt after)
    int32_t* d_ug = (int32_t*)L.chunks;
    int32_t* d_up = d_ug + nunits;
    int32_t* d_nch = d_up + nunits;
    int64_t* d_nel = (int64_t*)(d_nch + ((nunits + 1) & ~1));
    int32_t* d_err = (int32_t*)(d_nel + nunits);
    if ((int64_t)nunits * 24 + 64 > panel_chunk_cap(nnz) * (int64_t)sizeof(PanelChunk))
        return set_error("internal: panel build scratch"), MIPDHG_ERR_UNSUPPORTED;
    MIP_HIP(hipMemcpyAsync(d_ug, unit_group.data(), (size_t)nunits * 4, hipMemcpyHostToDevice, stream));
    MIP_HIP(hipMemcpyAsync(d_up, unit_panel.data(), (size_t)nunits * 4, hipMemcpyHostToDevice, stream));
    MIP_HIP(hipMemsetAsync(d_err, 0, 4, stream));
    MIP_HIP(hipMemsetAsync(L.counts, 0, (size_t)nseg * 4, stream));
    hipLaunchKernelGGL(k_seg_count, dim3(grid_for(nrows)), dim3(kBlock), 0, stream, rowptr, col, nrows,
                       (const int32_t*)L.row_group, (const PanelGroup*)L.groups, width, L.counts);
    const int ug = (nunits + 63) / 64;
    if (nunits > 0)
        hipLaunchKernelGGL((k_unit_chunks<false, V>), dim3(ug), dim3(64), 0, stream, (const PanelGroup*)L.groups,
                           (const int32_t*)d_ug, (const int32_t*)d_up, nunits, (const int32_t*)L.counts, d_nch, d_nel,
                           nullptr, nullptr, nullptr, nullptr, nullptr, (V*)nullptr, nullptr, nullptr, d_err);
    MIP_LAUNCH_CHECK();
    std::vector<int32_t> nch(nunits);
    std::vector<int64_t> nel(nunits);
    int32_t err = 0;
    if (nunits > 0) {
        MIP_HIP(hipMemcpyAsync(nch.data(), d_nch, (size_t)nunits * 4, hipMemcpyDeviceToHost, stream));
        MIP_HIP(hipMemcpyAsync(nel.data(), d_nel, (size_t)nunits * 8, hipMemcpyDeviceToHost, stream));
    }
    MIP_HIP(hipMemcpyAsync(&err, d_err, 4, hipMemcpyDeviceToHost, stream));
    MIP_HIP(hipStreamSynchronize(stream));
    if (err) return set_error("panel layout: a row has more than %d nonzeros in one panel", kPanelChunk),
                    MIPDHG_ERR_UNSUPPORTED;
    std::vector<int32_t> choff(nunits);
    std::vector<int64_t> eloff(nunits);
    int64_t tc = 0, te = 0;
    for (int u = 0; u < nunits; ++u) {
        choff[u] = (int32_t)tc;
        eloff[u] = te;
        tc += nch[u];
        te += nel[u];
    }
    if (tc > panel_chunk_cap(nnz) || te + kPanelChunk > panel_elem_cap(nnz))
        return set_error("panel layout: %lld chunks or %lld elements exceed the workspace's capacity",
                         (long long)tc, (long long)te),
               MIPDHG_ERR_UNSUPPORTED;
    L.nchunks = (int32_t)tc;
    L.nelem = te;
    // the fill pass writes the chunk array, which holds the unit tables: keep
    // those in the partial array meanwhile (at least as large, not yet in use)
    int32_t* s_ug = (int32_t*)L.partial;
    int32_t* s_up = s_ug + nunits;
    int32_t* s_choff = s_up + nunits;
    int64_t* s_eloff = (int64_t*)(s_choff + ((nunits + 1) & ~1));
    if ((int64_t)nunits * 24 + 64 > seg_cap * (int64_t)partial_elem_bytes)
        return set_error("internal: panel build scratch"), MIPDHG_ERR_UNSUPPORTED;
    MIP_HIP(hipMemcpyAsync(s_ug, unit_group.data(), (size_t)nunits * 4, hipMemcpyHostToDevice, stream));
    MIP_HIP(hipMemcpyAsync(s_up, unit_panel.data(), (size_t)nunits * 4, hipMemcpyHostToDevice, stream));
    MIP_HIP(hipMemcpyAsync(s_choff, choff.data(), (size_t)nunits * 4, hipMemcpyHostToDevice, stream));
    MIP_HIP(hipMemcpyAsync(s_eloff, eloff.data(), (size_t)nunits * 8, hipMemcpyHostToDevice, stream));
    if (nunits > 0)
        hipLaunchKernelGGL((k_unit_chunks<true, V>), dim3(ug), dim3(64), 0, stream, (const PanelGroup*)L.groups,
                           (const int32_t*)s_ug, (const int32_t*)s_up, nunits, (const int32_t*)L.counts, nullptr,
                           nullptr, (const int32_t*)s_choff, (const int64_t*)s_eloff, L.chunks, L.seg_off, L.seg_rid,
                           (V*)L.val, L.col, L.rid, (int32_t*)nullptr);
    MIP_LAUNCH_CHECK();
    // launch order: units with the most nonzeros first
    std::vector<int32_t> order(nunits);
    for (int u = 0; u < nunits; ++u) order[u] = u;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nel[a] > nel[b]; });
    std::vector<PanelUnit> units;
    for (int u : order)
        if (nel[u] > 0) units.push_back(PanelUnit{unit_group[u], unit_panel[u], choff[u], choff[u] + nch[u]});
    L.nunits = (int32_t)units.size();
    MIP_HIP(hipMemcpyAsync(L.units, units.data(), units.size() * sizeof(PanelUnit), hipMemcpyHostToDevice, stream));
    // scaled values, columns and rows in place; the counts become cursors
    MIP_HIP(hipMemsetAsync(L.counts, 0, (size_t)nseg * 4, stream));
    hipLaunchKernelGGL((k_panel_scatter<V>), dim3(grid_for(nrows)), dim3(kBlock), 0, stream, rowptr, col, val, d_self,
                       d_other, nrows, (const int32_t*)L.row_group, (const PanelGroup*)L.groups, width,
                       (const int32_t*)L.seg_off, (const uint16_t*)L.seg_rid, L.counts, (V*)L.val, L.col, L.rid);
    MIP_LAUNCH_CHECK();
    // partial sums of rows without nonzeros in a panel stay 0
    MIP_HIP(hipMemsetAsync(L.partial, 0, (size_t)nseg * partial_elem_bytes, stream));
    MIP_HIP(hipStreamSynchronize(stream));  // host vectors go out of scope
    return 0;
}

template int panel_build<double>(const std::vector<int32_t>&, int32_t, int32_t, int64_t, const int32_t*,
                                 const int32_t*, const double*, const double*, const double*, int, size_t,
                                 PanelLayout&, hipStream_t);
template int panel_build<float>(const std::vector<int32_t>&, int32_t, int32_t, int64_t, const int32_t*,
                                const int32_t*, const double*, const double*, const double*, int, size_t,
                                PanelLayout&, hipStream_t);
template int panel_build<uint16_t>(const std::vector<int32_t>&, int32_t, int32_t, int64_t, const int32_t*,
                                   const int32_t*, const double*, const double*, const double*, int, size_t,
                                   PanelLayout&, hipStream_t);

// ---------------------------------------------------------------------------
// row-panel layout (panel.h)
// ---------------------------------------------------------------------------
namespace {

// smallest and largest column below t0 of every row (none: lo > hi)
__global__ void k_row_span_below(const int32_t* rowptr, const int32_t* col, int32_t nrows, int32_t t0,
                                 int32_t* span) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * blockDim.x) {
        int32_t lo = 0x7fffffff, hi = -1;
        for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) {
            const int32_t c = col[k];
            if (c >= t0) continue;
            lo = c < lo ? c : lo;
            hi = c > hi ? c : hi;
        }
        span[2 * r] = lo;
        span[2 * r + 1] = hi;
    }
}

// every row's elements at their places: scaled value, place in the staged
// window or tail, row inside the chunk; an empty row's one element is 0
template <typename V>
__global__ void k_rowpanel_scatter(const int32_t* rowptr, const int32_t* col, const double* val, const double* d_self,
                                   const double* d_other, int32_t nrows, const int32_t* row_group,
                                   const RowPanelGroup* groups, int32_t t0, const int32_t* row_off,
                                   const uint16_t* row_rid, V* out, uint16_t* colv, uint16_t* rid) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * blockDim.x) {
        const RowPanelGroup g = groups[row_group[r]];
        const int64_t b = row_off[r];
        const uint16_t rr = row_rid[r];
        const int k0 = rowptr[r], k1 = rowptr[r + 1];
        if (k0 == k1) {
            out[b] = (V)0;
            colv[b] = 0;
            rid[b] = rr;
            continue;
        }
        const double ds = d_self[r];
        for (int k = k0; k < k1; ++k) {
            const int32_t cc = col[k];
            const double v = ds * val[k] * d_other[cc];  // the tile copies' expression
            const int64_t pos = b + (k - k0);
            if constexpr (sizeof(V) == 2) {
                out[pos] = f32_to_bf16_rne((float)v);
            } else {
                out[pos] = (V)v;
            }
            colv[pos] = (uint16_t)(cc < t0 ? cc - g.lo : g.ml + (cc - t0));
            rid[pos] = rr;
        }
    }
}

}  // namespace

template <typename V>
int rowpanel_build(const std::vector<int32_t>& rp, int32_t nrows, int32_t ncols, int64_t nnz, const int32_t* rowptr,
                   const int32_t* col, const double* val, const int32_t* rowptr_t, const int32_t* col_t,
                   const double* d_self, const double* d_other, int width, int cus, RowPanelLayout& L,
                   hipStream_t stream) {
    // --- the tail: the rows of the transpose that span more than half of its
    // columns and more than half a panel (the rows that couple everything,
    // such as linking rows) must be a final run of at most a quarter panel
    hipLaunchKernelGGL(k_row_span, dim3(grid_for(ncols)), dim3(kBlock), 0, stream, rowptr_t, col_t, ncols, L.span);
    MIP_LAUNCH_CHECK();
    std::vector<int32_t> span(2 * (size_t)std::max(nrows, ncols));
    MIP_HIP(hipMemcpyAsync(span.data(), L.span, 2 * (size_t)ncols * 4, hipMemcpyDeviceToHost, stream));
    MIP_HIP(hipStreamSynchronize(stream));
    int32_t t0 = ncols;
    for (int32_t i = 0; i < ncols; ++i)
        if (span[2 * i + 1] >= span[2 * i] &&
            (int64_t)span[2 * i + 1] - span[2 * i] + 1 > std::max<int64_t>(width / 2, nrows / 2)) {
            t0 = i;
            break;
        }
    if (ncols - t0 > width / 4)
        return set_error("row-panel layout: %d wide rows from row %d of A, more than a quarter panel (%d)", ncols - t0,
                         t0, width / 4),
               MIPDHG_ERR_UNSUPPORTED;
    t0 &= ~7;
    const int32_t tail = ncols - t0;
    const int32_t ml_max = (width - tail) & ~7;
    // --- every row's window below the tail
    hipLaunchKernelGGL(k_row_span_below, dim3(grid_for(nrows)), dim3(kBlock), 0, stream, rowptr, col, nrows, t0,
                       L.span);
    MIP_LAUNCH_CHECK();
    MIP_HIP(hipMemcpyAsync(span.data(), L.span, 2 * (size_t)nrows * 4, hipMemcpyDeviceToHost, stream));
    MIP_HIP(hipStreamSynchronize(stream));
    // --- groups of consecutive rows whose windows fit together
    std::vector<RowPanelGroup> groups;
    std::vector<int32_t> row_group(nrows), group_r0;
    int64_t glo = 0, ghi = -1;  // the open group's window (ghi < glo: none yet)
    auto flush = [&]() {
        RowPanelGroup g;
        if (ghi >= glo) {
            g.lo = (int32_t)(glo & ~7);
            g.ml = (int32_t)(((ghi - g.lo + 1) + 7) & ~7);
        } else {
            g.lo = 0;
            g.ml = 0;
        }
        groups.push_back(g);
    };
    for (int32_t r = 0; r < nrows; ++r) {
        const int32_t lo = span[2 * r], hi = span[2 * r + 1];
        if (r == 0) group_r0.push_back(0);
        if (hi >= lo) {
            if ((int64_t)hi - (lo & ~7) + 1 > ml_max)
                return set_error("row-panel layout: row %d spans %d columns below the tail, more than %d", r,
                                 hi - lo + 1, ml_max),
                       MIPDHG_ERR_UNSUPPORTED;
            const int64_t nlo = ghi >= glo ? std::min<int64_t>(glo, lo) : lo;
            const int64_t nhi = ghi >= glo ? std::max<int64_t>(ghi, hi) : hi;
            if (nhi - (nlo & ~7) + 1 > ml_max) {
                flush();
                group_r0.push_back(r);
                glo = lo;
                ghi = hi;
            } else {
                glo = nlo;
                ghi = nhi;
            }
        }
        row_group[r] = (int32_t)groups.size();
    }
    flush();
    group_r0.push_back(nrows);
    // --- units of about the same number of elements (an empty row counts one)
    int64_t total = 0;
    for (int32_t r = 0; r < nrows; ++r) total += std::max(1, rp[r + 1] - rp[r]);
    const int64_t target = std::max<int64_t>(4096, (total + 2 * (int64_t)cus - 1) / (2 * (int64_t)cus));
    std::vector<RowPanelUnit> units;
    std::vector<PanelChunk> chunks;
    std::vector<int32_t> row_off(nrows);
    std::vector<uint16_t> row_rid(nrows);
    int64_t e = 0;
    for (size_t gi = 0; gi + 1 < group_r0.size(); ++gi) {
        const int32_t r0 = group_r0[gi], r1 = group_r0[gi + 1];
        int32_t r = r0;
        while (r < r1) {  // one unit
            RowPanelUnit u;
            u.group = (int32_t)gi;
            u.c0 = (int32_t)chunks.size();
            int64_t acc = 0;
            int cnt = 0, row0 = -1;
            int64_t cstart = e;
            int nrow = 0;
            auto close = [&]() {
                if (cnt == 0) return;
                // a row-panel chunk's last field holds its row count
                chunks.push_back(PanelChunk{(int32_t)cstart, cnt, row0, nrow});
                nrow = 0;
                e = cstart + ((cnt + 7) & ~7);
                cnt = 0;
                row0 = -1;
            };
            while (r < r1 && (acc < target || r == r0)) {
                const int len = std::max(1, rp[r + 1] - rp[r]);
                if (len > kPanelChunk)
                    return set_error("row-panel layout: row %d has %d nonzeros, more than a chunk (%d)", r, len,
                                     kPanelChunk),
                           MIPDHG_ERR_UNSUPPORTED;
                if (cnt + len > kPanelChunk || (row0 >= 0 && r - row0 >= kRowPanelChunkRows)) close();
                if (row0 < 0) {
                    row0 = r;
                    cstart = e;
                }
                row_off[r] = (int32_t)(cstart + cnt);
                row_rid[r] = (uint16_t)(r - row0);
                ++nrow;
                cnt += len;
                acc += len;
                ++r;
                if (acc >= target) break;
            }
            close();
            u.c1 = (int32_t)chunks.size();
            units.push_back(u);
        }
    }
    if ((int64_t)units.size() > kRowPanelMaxUnits || (int64_t)chunks.size() > rowpanel_chunk_cap(nrows, nnz) ||
        e > rowpanel_elem_cap(nrows, nnz) || e >= INT32_MAX)
        return set_error("row-panel layout: %zu units, %zu chunks or %lld elements exceed the workspace's capacity",
                         units.size(), chunks.size(), (long long)e),
               MIPDHG_ERR_UNSUPPORTED;
    L.t0 = t0;
    L.tail = tail;
    L.ngroups = (int32_t)groups.size();
    L.nunits = (int32_t)units.size();
    L.nchunks = (int32_t)chunks.size();
    L.nelem = e;
    MIP_HIP(hipMemcpyAsync(L.groups, groups.data(), groups.size() * sizeof(RowPanelGroup), hipMemcpyHostToDevice,
                           stream));
    MIP_HIP(hipMemcpyAsync(L.units, units.data(), units.size() * sizeof(RowPanelUnit), hipMemcpyHostToDevice, stream));
    MIP_HIP(hipMemcpyAsync(L.chunks, chunks.data(), chunks.size() * sizeof(PanelChunk), hipMemcpyHostToDevice,
                           stream));
    MIP_HIP(hipMemcpyAsync(L.row_group, row_group.data(), (size_t)nrows * 4, hipMemcpyHostToDevice, stream));
    MIP_HIP(hipMemcpyAsync(L.row_off, row_off.data(), (size_t)nrows * 4, hipMemcpyHostToDevice, stream));
    MIP_HIP(hipMemcpyAsync(L.row_rid, row_rid.data(), (size_t)nrows * 2, hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL((k_rowpanel_scatter<V>), dim3(grid_for(nrows)), dim3(kBlock), 0, stream, rowptr, col, val,
                       d_self, d_other, nrows, (const int32_t*)L.row_group, (const RowPanelGroup*)L.groups, t0,
                       (const int32_t*)L.row_off, (const uint16_t*)L.row_rid, (V*)L.val, L.col, L.rid);
    MIP_LAUNCH_CHECK();
    MIP_HIP(hipStreamSynchronize(stream));  // host vectors go out of scope
    return 0;
}

#define MIP_ROWPANEL_INST(V)                                                                                       \
    template int rowpanel_build<V>(const std::vector<int32_t>&, int32_t, int32_t, int64_t, const int32_t*,         \
                                   const int32_t*, const double*, const int32_t*, const int32_t*, const double*,  \
                                   const double*, int, int, RowPanelLayout&, hipStream_t);
MIP_ROWPANEL_INST(double)
MIP_ROWPANEL_INST(float)
MIP_ROWPANEL_INST(uint16_t)
#undef MIP_ROWPANEL_INST

}  // namespace mip
