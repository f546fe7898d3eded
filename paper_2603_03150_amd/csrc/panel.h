// Panel layout of a matrix for an SpMV whose gathers are served from LDS.
//
// The rows are cut into groups of consecutive rows whose columns fall in a
// narrow span (a block of a block-structured matrix), or into groups of
// consecutive "wide" rows.  Each group's column span is cut into panels of at
// most kPanelBytes of the gathered vector; a unit is one (group, panel) pair.
// A workgroup per unit stages the panel's slice of the vector in LDS and
// streams the unit's nonzeros in row order -- value, a 16-bit column inside
// the panel, a 16-bit row index inside the chunk -- 8 per lane per load, in
// chunks of at most 512 nonzeros that end at a row end.  Each row's sum over
// the unit is written to a dense array of partial sums, panel-major within
// its group; a second kernel adds a row's partials in panel order.  The
// result does not depend on the launch: every sum is taken in a fixed order.
#pragma once
#include <stdint.h>

#include <vector>

#include "common.h"

namespace mip {

constexpr int kPanelBytes = 131072;       // LDS bytes of a staged panel
constexpr int kPanelChunk = 512;          // nonzeros per chunk (one wave, 8 per lane)
constexpr int kPanelBlock = 1024;         // threads per unit workgroup
constexpr int kPanelMaxGroupRows = 65535; // a 16-bit row index inside a chunk
constexpr int kPanelMaxUnits = 1 << 17;
constexpr int kPanelWideRow = 16;         // more panels: a wave adds the row's partials

template <typename T>
constexpr int panel_width() { return kPanelBytes / (int)sizeof(T); }

struct PanelGroup {
    int32_t r0, r1;     // rows [r0, r1)
    int32_t lo, np;     // first column of panel 0, number of panels
    int64_t seg_base;   // partial of row r, panel p: seg_base + p * (r1 - r0) + (r - r0)
};

struct PanelUnit {
    int32_t group, panel;
    int32_t c0, c1;     // chunks [c0, c1)
};

struct PanelChunk {
    int32_t start;      // first element (a multiple of 8)
    int32_t count;      // nonzeros (the chunk is padded to a multiple of 8)
    int32_t row0;       // first row (global)
    int32_t unit;       // the unit (panel layout); the row count (row-panel layout)
};

// Device arrays of the layout (inside the solver's workspace) and sizes.
struct PanelLayout {
    PanelGroup* groups;
    PanelUnit* units;
    PanelChunk* chunks;
    int32_t* row_group;   // [m]
    int32_t* wide_rows;   // [m] rows of groups with more than kPanelWideRow panels
    int32_t* counts;      // [segments] nonzeros per (row, panel) during the build
    int32_t* seg_off;     // [segments] first element of the row's part in the panel
    uint16_t* seg_rid;    // [segments] row index inside its chunk
    void* val;            // [elems] scaled values, type V
    uint16_t* col;        // [elems] column inside the panel
    uint16_t* rid;        // [elems] row inside the chunk
    void* partial;        // [segments] type T
    int32_t ngroups, nunits, nchunks, nwide;
    int64_t nseg, nelem;
};

// Capacities the workspace reserves for a matrix of nrows rows and nnz
// nonzeros (the layout is refused if it needs more).
inline int64_t panel_seg_cap(int64_t nrows, int64_t nnz) { return 5 * nrows + nnz + 1024; }
inline int64_t panel_chunk_cap(int64_t nnz) { return nnz / 64 + 2 * (int64_t)kPanelMaxUnits + 1; }
inline int64_t panel_elem_cap(int64_t nnz) { return nnz + 8 * panel_chunk_cap(nnz) + kPanelChunk; }

// Builds the layout of one matrix (row pointers rp on the host, the device
// CSR arrays, the row and column scaling) into the preallocated arrays of L:
// values d_self[r] * val * d_other[col] rounded to V, exactly as the tile
// copies.  Returns 0, MIPDHG_ERR_UNSUPPORTED if the matrix does not fit the
// layout's limits (a row part longer than a chunk, too many units or
// segments), or a HIP error.
template <typename V>
int panel_build(const std::vector<int32_t>& rp, int32_t nrows, int32_t ncols, int64_t nnz, const int32_t* rowptr,
                const int32_t* col, const double* val, const double* d_self, const double* d_other, int width,
                size_t partial_elem_bytes, PanelLayout& L, hipStream_t stream);

// ---------------------------------------------------------------------------
// Row-panel layout of A^T for the primal step: every row of A^T is summed
// whole inside one workgroup, so no partial sums are written.  The rows are
// cut into groups of consecutive rows whose columns, apart from a common tail
// [t0, ncols) (the rows of A that span the whole matrix, e.g. the linking rows
// of a block-angular LP), fall in a window [lo, lo + ml); a workgroup stages
// that window and the tail (together at most one panel) in LDS and the row's
// elements carry their column's place in it.  A group's rows are split into
// units (one workgroup each) of about the same number of nonzeros, units into
// chunks as in the panel layout; a row without nonzeros gets one element of
// value 0 so that its epilogue runs.
constexpr int kRowPanelMaxUnits = 2048;
constexpr int kRowPanelChunkRows = 128;  // rows of a chunk at most (their sums wait in LDS)

struct RowPanelGroup {
    int32_t lo, ml;     // staged window [lo, lo + ml), ml a multiple of 8; the tail follows at ml
};

struct RowPanelUnit {
    int32_t group;
    int32_t c0, c1;     // chunks [c0, c1)
};

struct RowPanelLayout {
    RowPanelGroup* groups;
    RowPanelUnit* units;
    PanelChunk* chunks;
    void* val;            // [elems] scaled values, type V
    uint16_t* col;        // [elems] place in the staged window and tail
    uint16_t* rid;        // [elems] row inside the chunk
    int32_t* row_group;   // [nrows] (build)
    int32_t* row_off;     // [nrows] first element of the row (build)
    uint16_t* row_rid;    // [nrows] (build)
    int32_t* span;        // [2 max(nrows, ncols)] (build)
    int32_t t0, tail;     // tail [t0, t0 + tail) of the gathered vector
    int32_t ngroups, nunits, nchunks;
    int64_t nelem;
};

inline int64_t rowpanel_chunk_cap(int64_t nrows, int64_t nnz) {
    return 2 * (nnz + nrows) / kPanelChunk + nrows / kRowPanelChunkRows + 2 * (int64_t)kRowPanelMaxUnits + 16;
}
inline int64_t rowpanel_elem_cap(int64_t nrows, int64_t nnz) {
    return nnz + nrows + 8 * rowpanel_chunk_cap(nrows, nnz) + kPanelChunk;
}

// Builds the row-panel layout of the matrix whose rows are rp/rowptr/col/val
// (A^T: nrows = n, ncols = m), from the host row pointers of both the matrix
// and its transpose (rp_t, the rows of A, used to find the tail): values
// d_self[r] * val * d_other[col] rounded to V, exactly as the tile copies.
// Returns 0, MIPDHG_ERR_UNSUPPORTED when the matrix does not have this
// structure (a row's window wider than the panel, a wide row of A outside a
// short final run, a row longer than a chunk), or a HIP error.
template <typename V>
int rowpanel_build(const std::vector<int32_t>& rp, int32_t nrows, int32_t ncols, int64_t nnz, const int32_t* rowptr,
                   const int32_t* col, const double* val, const int32_t* rowptr_t, const int32_t* col_t,
                   const double* d_self, const double* d_other, int width, int cus, RowPanelLayout& L,
                   hipStream_t stream);

}  // namespace mip
